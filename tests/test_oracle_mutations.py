"""Plant plausible mistakes in the oracle (on the CPU) and check that the pins catch them."""
import numpy as np
import pytest

import inputs as G
import oracle.lu as OL


def pins_pass() -> bool:
    """A compact run of the pins: known answer (square and tall), Wilkinson, zero pivot."""
    try:
        for (m, n), cfg in [((24, 24), dict(variant="rl", nb=5, inner=("rl", 2))),
                            ((30, 20), dict(variant="la", nb=4)),
                            ((20, 20), dict(variant="ll", nb=3))]:
            A, perm, L, U = G.known_answer(m, n, seed=m + n)
            F = A.copy()
            ipiv, info = OL.getrf(F, cfg["variant"], nb=cfg["nb"], inner=cfg.get("inner"))
            got = OL.permutation_of(ipiv, m)
            Lf, Uf = OL.unpack(F)
            k = min(m, n)
            if info != 0 or not np.array_equal(got[:k], perm[:k]) or not np.array_equal(Uf, U):
                return False
            if not np.array_equal(Lf, L[np.argsort(perm)[got]]):
                return False
        W = G.wilkinson_growth(12)
        F = W.copy()
        ipiv, _ = OL.getrf(F, "rl", nb=4)
        if ipiv != list(range(12)) or not np.array_equal(np.triu(F)[:, -1], 2.0 ** np.arange(12)):
            return False
        Z = G.zero_column(10, seed=1, col=4)
        F = Z.copy()
        _, info = OL.getrf(F, "rl", nb=3)
        return info == 5
    except Exception:
        return False


def test_unmutated_oracle_passes():
    assert pins_pass()


def _last_index_tie(x):
    a = np.abs(x)
    return int(len(a) - 1 - np.argmax(a[::-1]))


def _trsm_dropped_term(L, B, fl=None):
    X = B.copy()
    for r in range(1, L.shape[0]):
        X[r, :] = X[r, :] - L[r, :r - 1] @ X[:r - 1, :]
    return X


def _gemm_wrong_sign(C, A, B, fl=None):
    if C.size and A.shape[1]:
        C[...] = C + A @ B


def _gemm_drops_last_k(C, A, B, fl=None):
    if C.size and A.shape[1]:
        C[...] = C - A[:, :-1] @ B[:-1, :]


def _no_interchange(A, piv, row0=0):
    return None


def _unb_multiply_by_alpha(A, fl=None, info=None, col0=0):
    m, n = A.shape
    piv = []
    for c in range(min(m, n)):
        p = c + OL.iamax_first(A[c:, c])
        piv.append(p)
        OL.swap_rows(A, c, p)
        alpha = A[c, c]
        if alpha != 0:
            A[c + 1:, c] = A[c + 1:, c] * alpha
        A[c + 1:, c + 1:] = A[c + 1:, c + 1:] - np.outer(A[c + 1:, c], A[c, c + 1:])
    return piv


MUTATIONS = {
    "tie_takes_last_row": ("iamax_first", _last_index_tie),
    "trsm_drops_a_term": ("trsm_unit_lower", _trsm_dropped_term),
    "gemm_wrong_sign": ("gemm_update", _gemm_wrong_sign),
    "gemm_drops_last_k": ("gemm_update", _gemm_drops_last_k),
    "interchanges_skipped": ("apply_interchanges", _no_interchange),
    "rl1_multiplies": ("lu_unb", _unb_multiply_by_alpha),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, monkeypatch):
    attr, bad = MUTATIONS[name]
    monkeypatch.setattr(OL, attr, bad)
    assert not pins_pass(), f"pins did not catch: {name}"
