"""Pins of the CPU oracle against facts fixed outside of it (no GPU needed).

Each pin is chosen so that a plausible mistake in the oracle (a dropped term, a
wrong sign or index, a transposed operand, a wrong tie rule, a skipped
interchange) fails at least one of them; test_oracle_mutations.py plants such
mistakes and checks that they are caught.
"""
from fractions import Fraction
from itertools import permutations

import numpy as np
import pytest
import scipy.linalg as sla

import inputs as G
import oracle as O
from oracle import invariants as I


# ----------------------------------------------------------------- helpers
def det_leibniz(M):
    """Determinant by the permutation expansion (independent of elimination)."""
    k = len(M)
    if k == 0:
        return Fraction(1)
    total = Fraction(0)
    for perm in permutations(range(k)):
        sgn = 1
        for a in range(k):
            for b in range(a + 1, k):
                if perm[a] > perm[b]:
                    sgn = -sgn
        prod = Fraction(1)
        for r in range(k):
            prod *= M[r][perm[r]]
            if prod == 0:
                break
        total += sgn * prod
    return total


def sub(B, rows, cols):
    return [[B[r][c] for c in cols] for r in rows]


def frac(A):
    return np.array([[Fraction(int(x)) if float(x).is_integer() else Fraction(float(x)) for x in row]
                     for row in A], dtype=object)


def minors_lu(B):
    """L and U of B = L U from ratios of minors (Gantmacher), B already permuted."""
    m, n = len(B), len(B[0])
    k = min(m, n)
    U = [[Fraction(0)] * n for _ in range(k)]
    L = [[Fraction(0)] * k for _ in range(m)]
    lead = [det_leibniz(sub(B, range(i), range(i))) for i in range(k + 1)]
    for i in range(k):
        for j in range(i, n):
            U[i][j] = det_leibniz(sub(B, range(i + 1), list(range(i)) + [j])) / lead[i]
    for j in range(k):
        L[j][j] = Fraction(1)
        for i in range(j + 1, m):
            L[i][j] = det_leibniz(sub(B, list(range(j)) + [i], range(j + 1))) / lead[j + 1]
    return L, U


def check_pivot_rule(Ahat, ipiv):
    """At step c the chosen row maximises |Schur complement| (first on ties),
    with the candidates computed from determinants, not by elimination."""
    B = [list(r) for r in Ahat]
    m, n = len(B), len(B[0])
    for c in range(min(m, n)):
        den = det_leibniz(sub(B, range(c), range(c)))
        cand = [abs(det_leibniz(sub(B, list(range(c)) + [i], range(c + 1))) / den)
                for i in range(c, m)]
        best = max(cand)
        assert ipiv[c] == c + cand.index(best), (c, ipiv, cand)
        B[c], B[ipiv[c]] = B[ipiv[c]], B[c]


CONFIGS = [
    dict(variant="rl", nb=1), dict(variant="rl", nb=2), dict(variant="rl", nb=3, inner=("rl", 2)),
    dict(variant="rl", nb=4, inner=("ll", 2)), dict(variant="ll", nb=1), dict(variant="ll", nb=2),
    dict(variant="ll", nb=3, lazy=False), dict(variant="ll", nb=3, inner=("rl", 2)),
    dict(variant="la", nb=1), dict(variant="la", nb=2), dict(variant="la", nb=3, inner=("ll", 2)),
    dict(variant="la", nb=100),
]


def run(A, variant, nb=None, schedule=None, inner=None, lazy=True, fl=None):
    F = A.copy()
    ipiv, info = O.getrf(F, variant, nb=nb, schedule=schedule, inner=inner, fl=fl, lazy=lazy)
    return F, ipiv, info


# ----------------------------------------------------------------- exact brute force
@pytest.mark.parametrize("shape", [(4, 4), (5, 5), (6, 4), (4, 6), (5, 3), (1, 1), (1, 4), (4, 1)])
@pytest.mark.parametrize("seed", range(3))
def test_exact_minors_and_pivot_rule(shape, seed):
    m, n = shape
    # small integers in [-2, 2]: exact ties between pivot candidates are common
    for s in range(seed * 50, seed * 50 + 50):
        A = frac(G.small_int_matrix(m, n, seed=s, lo=-2, hi=2))
        F, ipiv, info = run(A, "rl", nb=1)
        if info == 0:
            break
    assert info == 0
    check_pivot_rule(A, ipiv)
    perm = O.permutation_of(ipiv, m)
    B = A[perm, :]
    Lm, Um = minors_lu(B.tolist())
    L, U = O.unpack(F)
    assert all(L[i, j] == Lm[i][j] for i in range(m) for j in range(min(m, n)))
    assert all(U[i, j] == Um[i][j] for i in range(min(m, n)) for j in range(n))
    for cfg in CONFIGS:
        F2, ipiv2, info2 = run(A, **cfg)
        assert ipiv2 == ipiv, cfg
        assert all(x == y for x, y in zip(F2.ravel(), F.ravel())), cfg
    for t in range(3):
        sch = G.random_schedule(min(m, n), seed=t, max_b=3)
        for v in ("rl", "ll", "la"):
            F2, ipiv2, _ = run(A, v, schedule=sch)
            assert ipiv2 == ipiv and all(x == y for x, y in zip(F2.ravel(), F.ravel())), (v, sch)


def test_exact_ties_take_first_row():
    # column 0 candidates are 2, -2, 2: the first row (0) wins, no interchange
    A = frac(np.array([[2, 1, 0], [-2, 3, 1], [2, 0, 5]]))
    F, ipiv, _ = run(A, "rl", nb=1)
    assert ipiv[0] == 0
    A = frac(np.array([[1, 1, 0], [-2, 3, 1], [2, 0, 5]]))
    F, ipiv, _ = run(A, "rl", nb=1)
    assert ipiv[0] == 1          # |-2| ties |2|; row 1 comes first


# ----------------------------------------------------------------- Wilkinson growth
@pytest.mark.parametrize("n", [3, 8, 40, 53])
@pytest.mark.parametrize("cfg", CONFIGS)
def test_wilkinson_growth_matrix(n, cfg):
    W = G.wilkinson_growth(n)
    F, ipiv, info = run(W, **cfg)
    assert info == 0
    assert ipiv == list(range(n))                       # every column is a tie: P = I
    L, U = O.unpack(F)
    assert np.array_equal(L, np.eye(n) - np.tril(np.ones((n, n)), -1))
    expect_last = 2.0 ** np.arange(n)                   # U(i, n-1) = 2^i exactly
    assert np.array_equal(U[:, n - 1], expect_last)
    assert np.array_equal(U[:, :n - 1], np.eye(n)[:, :n - 1])


# ----------------------------------------------------------------- known answer
@pytest.mark.parametrize("shape", [(16, 16), (64, 64), (40, 25), (25, 40), (1, 1), (7, 1), (1, 7)])
@pytest.mark.parametrize("cfg", CONFIGS + [dict(variant="rl", nb=8, inner=("rl", 3))])
def test_known_answer_exact(shape, cfg):
    m, n = shape
    A, perm, L, U = G.known_answer(m, n, seed=m * 100 + n)
    F, ipiv, info = run(A, **cfg)
    assert info == 0
    k = min(m, n)
    got = O.permutation_of(ipiv, m)
    # the first k rows are the pivots; rows below keep whatever order the
    # interchanges left them in, and L's rows follow them
    assert np.array_equal(got[:k], perm[:k])
    inv = np.argsort(perm)
    Lf, Uf = O.unpack(F)
    assert np.array_equal(Uf, U)
    assert np.array_equal(Lf, L[inv[got]])


def test_zero_pivot_info_and_continues():
    for col in (0, 5, 11):
        A = G.zero_column(12, seed=4, col=col)
        for cfg in CONFIGS:
            F, ipiv, info = run(A, **cfg)
            assert info == col + 1, (cfg, info)
            pc = I.postcondition(A, F, ipiv)
            assert pc["rel_frob"] == 0.0


# ----------------------------------------------------------------- flop model
def test_flop_count_closed_forms():
    for n in (1, 2, 3, 10, 57):
        assert 6 * O.flops_lu_exact(n, n) == 4 * n ** 3 - 3 * n ** 2 - n   # 2n^3/3 - n^2/2 - n/6
    for (m, n) in ((50, 20), (20, 50), (31, 31)):
        k = min(m, n)
        # leading terms m n^2 - n^3/3 (m >= n); exact lower-order terms
        exact = sum((m - c - 1) * (1 + 2 * (n - c - 1)) for c in range(k))
        assert O.flops_lu_exact(m, n) == exact
    n = 3000
    assert abs(O.flops_lu_exact(n, n) / (2 * n ** 3 / 3) - 1) < 1e-3


@pytest.mark.parametrize("variant", ["rl", "ll", "la"])
def test_flop_counter_matches_model(variant):
    n, b = 96, 8
    A = G.uniform01(n, seed=1)
    fl = O.Flops()
    run(A, variant, nb=b, fl=fl)
    # every variant performs the same multiply-adds, only reordered
    assert fl.total == O.flops_lu_exact(n, n)


def test_flop_share_of_leading_iterations():
    # Section 3.1: first 25% / 50% / 75% of RL iterations hold ~58%, 87.5%, >98%
    n = 400
    A = G.uniform01(n, seed=2)
    fl = O.Flops()
    seen = []
    O.lu_blk_rl(A, nb=1, fl=fl, on_iter=lambda k, j, A_, p: seen.append(fl.total))
    total = seen[-1]
    f25, f50, f75 = (seen[int(n * f) - 1] / total for f in (0.25, 0.5, 0.75))
    assert abs(f25 - 0.58) < 0.01 and abs(f50 - 0.875) < 0.01 and f75 > 0.98


@pytest.mark.parametrize("n,b", [(480, 16), (512, 32)])
def test_panel_flop_share(n, b):
    # Section 3.1: all panels cost about n^2 b / 2, a share of 3b/(4n)
    A = G.uniform01(n, seed=3)
    fl = O.Flops()
    O.lu_blk_rl(A, nb=b, fl=fl)
    assert abs(fl.panel / (n * n * b / 2) - 1) < 0.06
    assert abs(fl.panel / fl.total / (3 * b / (4 * n)) - 1) < 0.06
    assert fl.total == O.flops_lu_exact(n, n)


def test_panel_share_quoted_case():
    # "less than 2%" at n = 10,000, b_o = 256 (Section 3.1, trace discussion)
    assert 3 * 256 / (4 * 10000) < 0.02


# ----------------------------------------------------------------- library cross-check
@pytest.mark.parametrize("n", [64, 200, 333])
@pytest.mark.parametrize("cfg", [dict(variant="rl", nb=16), dict(variant="la", nb=32, inner=("rl", 8)),
                                 dict(variant="ll", nb=24)])
def test_against_lapack_getrf(n, cfg):
    A = G.uniform01(n, seed=n)
    lu, piv = sla.lu_factor(A)
    F, ipiv, info = run(A, **cfg)
    assert info == 0
    assert np.array_equal(np.array(ipiv), piv)
    scale = np.abs(lu).max()
    assert np.abs(F - lu).max() <= 1e-13 * scale * n ** 0.5


def test_spd_workload_makes_no_interchange():
    A = G.spd_bbt(256, seed=0)
    F, ipiv, info = run(A, "rl", nb=32)
    assert ipiv == list(range(256))
    pc = I.postcondition(A, F, ipiv)
    assert pc["rel_frob"] <= 1e-15


def test_uniform_workload_makes_many_interchanges():
    A = G.uniform01(256, seed=0)
    F, ipiv, _ = run(A, "rl", nb=32)
    assert sum(p != i for i, p in enumerate(ipiv)) > 200


# ----------------------------------------------------------------- invariants
def _collect(variant, A, nb=None, schedule=None, inner=None, lazy=True):
    F = A.copy()
    errs = []
    sched = O.schedule_from(min(A.shape), nb, schedule)

    def cb(k, j, S, ipiv, pend=None):
        if variant == "rl":
            errs.append(I.check_rl(A, S, ipiv, j))
        elif variant == "ll":
            errs.append(I.check_ll(A, S, ipiv, j, lazy))
        else:
            bp = sched[k + 1] if k + 1 < len(sched) else 0
            errs.append(I.check_la(A, S, ipiv, pend, j, bp))

    ipiv, info = O.getrf(F, variant, nb=nb, schedule=schedule, inner=inner, on_iter=cb, lazy=lazy)
    return F, ipiv, errs


@pytest.mark.parametrize("variant", ["rl", "ll", "la"])
@pytest.mark.parametrize("shape", [(48, 48), (60, 37), (37, 60)])
def test_loop_invariant_every_iteration_fp64(variant, shape):
    A = G.uniform01(*shape, seed=9)
    for sched in (None, G.random_schedule(min(shape), seed=1, max_b=9)):
        F, ipiv, errs = _collect(variant, A, nb=8 if sched is None else None, schedule=sched)
        assert len(errs) == len(O.schedule_from(min(shape), 8, sched))
        assert max(errs) < 1e-14
        assert I.postcondition(A, F, ipiv)["rel_frob"] < 1e-14


@pytest.mark.parametrize("variant", ["rl", "ll", "la"])
def test_loop_invariant_exact(variant):
    A = frac(G.small_int_matrix(6, 6, seed=21, lo=-4, hi=4))
    for lazy in (True, False):
        F, ipiv, errs = _collect(variant, A, schedule=[2, 1, 3], lazy=lazy)
        assert errs and all(e == 0.0 for e in errs)


def test_invariant_checker_detects_a_wrong_state():
    A = G.uniform01(20, seed=5)
    F, ipiv, errs = _collect("rl", A, nb=5)
    j = 20
    assert I.check_rl(A, F, ipiv, j) < 1e-14
    G2 = F.copy()
    G2[7, 3] += 1e-6
    assert I.check_rl(A, G2, ipiv, j) > 1e-9
    bad = list(ipiv)
    bad[4], bad[5] = bad[5], bad[4]
    assert I.check_rl(A, F, bad, j) > 1e-9 or bad == ipiv


def test_iters_limit_states_satisfy_invariants():
    A = G.uniform01(30, seed=6)
    sched = O.schedule_from(30, 7)
    for s in range(len(sched) + 1):
        F = A.copy()
        ipiv, _ = O.lu_blk_rl(F, nb=7, iters_limit=s)
        assert I.check_rl(A, F, ipiv, sum(sched[:s])) < 1e-14
        F = A.copy()
        ipiv, _ = O.lu_blk_ll(F, nb=7, iters_limit=s)
        assert I.check_ll(A, F, ipiv, sum(sched[:s])) < 1e-14
        F = A.copy()
        ipiv, _ = O.lu_blk_la(F, nb=7, iters_limit=s)
        j = sum(sched[:s])
        bp = sched[s] if s < len(sched) else 0
        done, pend = ipiv[:j], [p - j for p in ipiv[j:]]
        assert I.check_la(A, F, done, pend, j, bp) < 1e-14


# ----------------------------------------------------------------- triangular solves
@pytest.mark.parametrize("uplo", ["L", "U"])
@pytest.mark.parametrize("diag", ["U", "N"])
def test_trsm_exact_known_solution(uplo, diag):
    rng = np.random.default_rng(1)
    n, k = 12, 5
    T = rng.integers(-7, 8, (n, n)) / 8.0
    d = 2.0 ** rng.integers(-2, 3, n) * rng.choice([-1, 1], n)
    T[np.arange(n), np.arange(n)] = d
    Tt = np.tril(T) if uplo == "L" else np.triu(T)
    if diag == "U":
        Tt = Tt.copy()
        Tt[np.arange(n), np.arange(n)] = 1.0
    X = rng.integers(-9, 10, (n, k)).astype(float)
    B = Tt @ X                                   # exact: dyadic products, small sums
    Y = O.trsm(T, B, uplo, diag)                 # reads only the named triangle
    assert np.array_equal(Y, X)


def test_trsm_config0_operand_residual():
    T = G.tri_operand(256, seed=0)
    rng = np.random.default_rng(2)
    B = rng.standard_normal((256, 8))
    for uplo, TT in (("L", T), ("U", np.ascontiguousarray(T.T))):
        X = O.trsm(TT, B, uplo, "N")
        Tt = np.tril(TT) if uplo == "L" else np.triu(TT)
        R = Tt @ X - B
        # off-diagonal entries ~16 over a diagonal in [1, 2]: the solution grows
        # to ~1e200, so the backward error uses infinity norms (no squares)
        inf = lambda M: np.abs(M).sum(axis=1).max()
        assert inf(R) / (inf(Tt) * inf(X)) < 256 * np.finfo(float).eps


def test_getrs_exact_known_solution():
    A, perm, L, U = G.known_answer(20, 20, seed=8)
    x = np.random.default_rng(3).integers(-5, 6, (20, 3)).astype(float)
    b = A @ x
    F, ipiv, _ = run(A, "rl", nb=6)
    assert np.array_equal(O.getrs(F, ipiv, b), x)


def test_schedule_rules():
    assert O.schedule_from(10, 4) == [4, 4, 2]
    assert O.schedule_from(10, 1) == [1] * 10
    assert O.schedule_from(10, 99) == [10]
    assert O.schedule_from(10, schedule=[3, 3, 9]) == [3, 3, 4]
    with pytest.raises(ValueError):
        O.schedule_from(10, schedule=[3, 3])
