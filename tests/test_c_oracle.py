"""Pins of the plain C oracle (oracle/lu_blk.c): same facts as the Python oracle's,
plus agreement with the Python oracle.  CPU only."""
import numpy as np
import pytest

import inputs as G
import oracle as O
from oracle import c_oracle as C


@pytest.fixture(scope="module", autouse=True)
def _built():
    C.build(force=False)


@pytest.mark.parametrize("nb", [1, 5, 64])
@pytest.mark.parametrize("shape", [(64, 64), (50, 30), (30, 50)])
def test_known_answer_exact(shape, nb):
    m, n = shape
    A, perm, L, U = G.known_answer(m, n, seed=7)
    F = A.copy()
    ipiv, info = C.dgetrf_rl(F, nb)
    assert info == 0
    got = O.permutation_of(list(ipiv - 1), m)
    k = min(m, n)
    assert np.array_equal(got[:k], perm[:k])
    Lf, Uf = O.unpack(F)
    assert np.array_equal(Uf, U)
    assert np.array_equal(Lf, L[np.argsort(perm)[got]])


def test_wilkinson():
    W = G.wilkinson_growth(50)
    ipiv, info = C.dgetrf_rl(W, 8)
    assert list(ipiv) == list(range(1, 51))
    assert np.array_equal(np.triu(W)[:, -1], 2.0 ** np.arange(50))


def test_zero_pivot():
    Z = G.zero_column(16, seed=2, col=9)
    ipiv, info = C.dgetrf_rl(Z, 4)
    assert info == 10


@pytest.mark.parametrize("n,nb", [(200, 16), (257, 32)])
def test_agrees_with_python_oracle(n, nb):
    A = G.uniform01(n, seed=n)
    F = A.copy()
    ipiv, info = C.dgetrf_rl(F, nb)
    P = A.copy()
    ip2, _ = O.getrf(P, "rl", nb=nb)
    assert np.array_equal(ipiv - 1, np.array(ip2))
    assert np.abs(F - P).max() <= 1e-13 * np.abs(P).max()
