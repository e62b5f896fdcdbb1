"""Negative pins of the loop-invariant checkers (LA and LL; RL is pinned in
test_oracle_pins.py) and of the LU-IR -> GMRES-IR switch of the refinement
oracle.

The GPU `iters_limit` parity rests on these checkers (the invariants derived
for Fig. "LU" and Fig. "LU_la_blk", Sections 3.1 and 3.2, and for the
left-looking variant of Section 4.2), so each relation must be shown to be
tested, not only satisfied by correct states:

  * a state with one entry corrupted in any block of the partition fails;
  * for every relation there is a corrupted specification (A_hat changed in
    the one block of P A_hat that only that relation reads) that fails, so a
    checker that dropped that relation (a planted mutation, below) lets it
    pass and is caught.
"""
import numpy as np
import pytest

import inputs as G
import oracle as O
from oracle import invariants as I
from oracle import refine as R

BAD = 1e-9     # a corrupted state must be reported at least this far off
GOOD = 1e-14   # a correct FP64 state of these sizes stays below this


def unpermute(Ap, ipiv):
    """A_hat with P A_hat = Ap (the sequential interchanges undone in reverse)."""
    A = Ap.copy()
    for c in reversed(range(len(ipiv))):
        p = ipiv[c]
        if p != c:
            A[[c, p], :] = A[[p, c], :]
    return A


def permute(A, ipiv):
    Ap = A.copy()
    O.apply_interchanges(Ap, ipiv)
    return Ap


def la_state(m=40, n=36, nb=7, s=2, seed=3):
    """Oracle LA state after s loop bodies: (A_hat, state, done, pend, j, bp)."""
    A = G.uniform01(m, n, seed=seed)
    sched = O.schedule_from(min(m, n), nb)
    F = A.copy()
    ipiv, _ = O.lu_blk_la(F, nb=nb, iters_limit=s)
    j = sum(sched[:s])
    bp = sched[s] if s < len(sched) else 0
    done, pend = ipiv[:j], [p - j for p in ipiv[j:]]
    return A, F, done, pend, j, bp


def ll_state(lazy, m=40, n=36, nb=7, s=2, seed=4):
    A = G.uniform01(m, n, seed=seed)
    sched = O.schedule_from(min(m, n), nb)
    F = A.copy()
    ipiv, _ = O.lu_blk_ll(F, nb=nb, iters_limit=s, lazy=lazy)
    return A, F, ipiv, sum(sched[:s])


# Blocks of the LA partition at the top of the loop: (rows, cols) slices.
def la_blocks(m, n, j, bp):
    return {
        "TL": (slice(0, j), slice(0, j)),
        "TR": (slice(0, j), slice(j, n)),
        "BL": (slice(j, m), slice(0, j)),
        "P": (slice(j, m), slice(j, j + bp)),
        "R": (slice(j, m), slice(j + bp, n)),
    }


def ll_blocks(m, n, j):
    return {
        "TL": (slice(0, j), slice(0, j)),
        "BL": (slice(j, m), slice(0, j)),
        "TR": (slice(0, j), slice(j, n)),
        "BR": (slice(j, m), slice(j, n)),
    }


def poke(X, blk, delta=1e-6):
    """X with one entry in the middle of block blk moved by delta * max|X|."""
    rows, cols = blk
    r = (rows.start + rows.stop) // 2
    c = (cols.start + cols.stop) // 2
    Y = X.copy()
    Y[r, c] += delta * np.abs(X).max()
    return Y


def la_pins_pass(check) -> bool:
    """Every LA relation is tested by `check` (the checker under test)."""
    A, F, done, pend, j, bp = la_state()
    m, n = A.shape
    if not check(A, F, done, pend, j, bp) < GOOD:
        return False
    Ap = permute(A, done)
    for name, blk in la_blocks(m, n, j, bp).items():
        if not check(A, poke(F, blk), done, pend, j, bp) > BAD:          # wrong state
            return False
        if not check(unpermute(poke(Ap, blk), done), F, done, pend, j, bp) > BAD:   # wrong spec
            return False
    # a pending interchange changed, and an interchange already made changed
    bad = list(pend)
    bad[1] = bad[0] if bad[1] != bad[0] else bad[1] + 1
    if not check(A, F, done, bad, j, bp) > BAD:
        return False
    bad = list(done)
    bad[2] = 2 if bad[2] != 2 else 3
    return check(A, F, bad, pend, j, bp) > BAD


def ll_pins_pass(check) -> bool:
    for lazy in (True, False):
        A, F, ipiv, j = ll_state(lazy)
        m, n = A.shape
        if not check(A, F, ipiv, j, lazy) < GOOD:
            return False
        Ap = permute(A, ipiv)
        for name, blk in ll_blocks(m, n, j).items():
            if not check(A, poke(F, blk), ipiv, j, lazy) > BAD:
                return False
            if name in ("TL", "BL"):       # relations on P A_hat's left columns
                spec = unpermute(poke(Ap, blk), ipiv)
            elif lazy:                     # the untouched right part is A_hat itself
                spec = poke(A, blk)
            else:                          # eager: the permuted A_hat
                spec = unpermute(poke(Ap, blk), ipiv)
            if not check(spec, F, ipiv, j, lazy) > BAD:
                return False
        # the other form of the right part is a different state once rows moved
        moved = any(p != c for c, p in enumerate(ipiv))
        if moved and not check(A, F, ipiv, j, not lazy) > BAD:
            return False
    return True


def test_la_checker_accepts_every_oracle_state():
    for s in range(0, 6):
        A, F, done, pend, j, bp = la_state(s=s)
        assert I.check_la(A, F, done, pend, j, bp) < GOOD


def test_la_checker_rejects_each_corrupted_block():
    assert la_pins_pass(I.check_la)


def test_ll_checker_rejects_each_corrupted_block_lazy_and_eager():
    assert ll_pins_pass(I.check_ll)


def test_states_make_interchanges():
    # the pins mean something only if rows actually moved in both states
    A, F, done, pend, j, bp = la_state()
    assert sum(p != c for c, p in enumerate(done)) >= 3
    assert sum(p != c for c, p in enumerate(pend)) >= 3
    for lazy in (True, False):
        _, _, ipiv, _ = ll_state(lazy)
        assert sum(p != c for c, p in enumerate(ipiv)) >= 3


def dropping(check, k):
    """Planted mutation: `check` with its k-th relation (0-based) always satisfied."""
    def mutant(*args, **kw):
        calls = [0]
        orig = I._rel

        def rel(X, Y, scale):
            i = calls[0]
            calls[0] += 1
            return 0.0 if i == k else orig(X, Y, scale)

        I._rel = rel
        try:
            return check(*args, **kw)
        finally:
            I._rel = orig
    return mutant


@pytest.mark.parametrize("k", range(5))   # TL, TR, BL, P, R
def test_la_checker_without_a_relation_is_caught(k):
    assert not la_pins_pass(dropping(I.check_la, k))


@pytest.mark.parametrize("k", range(3))   # TL, BL, right part
def test_ll_checker_without_a_relation_is_caught(k):
    assert not ll_pins_pass(dropping(I.check_ll, k))


# ---------------------------------------------------------------- auto switch
# A = diag(a), M^{-1} = I, b = (1, 1e-3): after x_0 = b the LU-IR residual is
# r_i = (1 - a)^(i+1) * b componentwise, a closed form.  With contractions
# 0.1 and 0.6 the first component dominates until i = 3 and the second from
# i = 4 on, so berr_4 / berr_3 is about 0.6: the correction x_3 -> x_4 is the
# first that fails to halve the backward error, and x_4 -> x_5 must be the
# first GMRES correction.  GMRES on diag(a) d = r is exact after 2 steps
# (two distinct eigenvalues).
A_SW = np.diag([0.9, 0.4])
B_SW = np.array([1.0, 1e-3])


def closed_form_berrs(count):
    a = np.diag(A_SW)
    out = []
    for i in range(count):
        r = (1.0 - a) ** (i + 1) * B_SW
        x = (B_SW - r) / a
        den = np.abs(A_SW).sum(axis=1).max() * np.abs(x).max() + np.abs(B_SW).max()
        out.append(float(np.abs(r).max() / den))
    return out


def ident(r):
    return np.array(r, dtype=float)


def test_auto_switch_happens_at_the_first_correction_that_does_not_halve():
    expect = closed_form_berrs(5)
    ratios = [expect[i] / expect[i - 1] for i in range(1, 5)]
    assert all(q < 0.5 for q in ratios[:3]) and ratios[3] > 0.5   # the script itself
    # LU-IR alone follows the closed form
    _, outer, inner, berrs = R.refine(A_SW, B_SW, ident, tol=1e-30, max_outer=4, solver="lu")
    assert outer == -1 and inner == 0
    np.testing.assert_allclose(berrs, expect, rtol=1e-12)
    # auto: no GMRES step through x_4 ...
    _, outer, inner, berrs = R.refine(A_SW, B_SW, ident, tol=1e-30, max_outer=4, solver="auto")
    assert inner == 0
    np.testing.assert_allclose(berrs, expect, rtol=1e-12)
    # ... and the correction from x_4 is GMRES (2 steps, exact)
    _, outer, inner, berrs = R.refine(A_SW, B_SW, ident, tol=1e-15, max_outer=6, solver="auto")
    assert inner == 2 and outer == 5
    np.testing.assert_allclose(berrs[:5], expect, rtol=1e-12)
    assert berrs[5] < 1e-15


@pytest.mark.parametrize("ratio,first_gmres", [(0.05, 1), (0.7, None)])
def test_auto_switch_ratio_moves_the_switch(ratio, first_gmres):
    # a stricter ratio switches after the first correction (0.1 > 0.05); a
    # looser one never switches within 6 corrections (every ratio <= 0.6)
    _, outer, inner, berrs = R.refine(A_SW, B_SW, ident, tol=1e-30, max_outer=6, solver="auto",
                                      switch_ratio=ratio)
    if first_gmres is None:
        assert inner == 0
    else:
        _, _, inner_before, _ = R.refine(A_SW, B_SW, ident, tol=1e-30, max_outer=first_gmres,
                                         solver="auto", switch_ratio=ratio)
        assert inner_before == 0 and inner > 0
