"""GPU parity of the look-ahead LU with early termination of the panel
(mlu_dgetrf_et, Section 4.2): the realized panel widths are a schedule, and
the factorization must be the oracle's look-ahead LU with that schedule and a
left-looking inner LU of the same block size.

Bars: pivots identical; factors within 1e-12 * max|F_oracle| (rounding order
differs); known-answer inputs bit-exact.  The stop decision is timing
dependent under force="signal"; force="always" (stop after the first block of
every look-ahead panel) and "never" exercise both paths deterministically, by
a flag set from the host side of the call, never by a fault.
"""
import numpy as np
import pytest
import torch

import inputs as G
import oracle as O
from paper_1611_06365_amd import mlu

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    mlu.load()
    yield
    torch.cuda.synchronize()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def run_et(A, nb, bi, force, min_width=0):
    dA = torch.from_numpy(np.ascontiguousarray(A)).to(DEV)
    ipiv, info, widths = mlu.getrf_et(dA, nb=nb, nb_inner=bi, force=force, min_width=min_width)
    k = min(A.shape)
    return host(dA), (host(ipiv)[:k] - 1).tolist(), int(host(info)[0]), widths


def check_widths(widths, mn, nb, bi):
    assert sum(widths) == mn and all(w >= 1 for w in widths)
    assert widths[0] == min(nb, mn)
    j = widths[0]
    for w in widths[1:]:
        planned = min(nb, mn - j)
        assert w <= planned and (w % bi == 0 or w == planned), (w, planned)
        j += w


@pytest.mark.parametrize("force", ["always", "never", "signal"])
@pytest.mark.parametrize("shape,nb,bi", [((600, 600), 64, 16), ((700, 500), 96, 16), ((450, 620), 64, 8),
                                         ((1100, 1100), 256, 16)])
def test_et_matches_oracle_with_realized_schedule(force, shape, nb, bi):
    m, n = shape
    A = G.uniform01(m, n, seed=m + n) if m != n else G.uniform01(m, seed=m)
    F, piv, info, widths = run_et(A, nb, bi, force)
    mn = min(m, n)
    check_widths(widths, mn, nb, bi)
    if force == "always":   # every look-ahead panel stops after its first block
        j = widths[0]
        for w in widths[1:]:
            assert w == min(bi, nb, mn - j)
            j += w
    if force == "never":
        assert widths == O.schedule_from(mn, nb)
    R = A.copy()
    opiv, oinfo = O.getrf(R, "la", schedule=widths, inner=("ll", bi))
    print(f"ET {force} {shape} nb={nb}: {len(widths)} panels, widths {widths[:8]}...", flush=True)
    assert info == oinfo == 0
    assert piv == opiv
    assert np.abs(F - R).max() <= 1e-12 * np.abs(R).max()


@pytest.mark.parametrize("force", ["always", "signal"])
def test_et_known_answer_exact(force):
    A, perm, L, U = G.known_answer(520, 520, seed=9)
    F, piv, info, widths = run_et(A, 128, 16, force)
    R = A.copy()
    opiv, _ = O.getrf(R, "la", schedule=widths, inner=("ll", 16))
    assert info == 0 and piv == opiv
    assert np.array_equal(F, R)
    assert np.array_equal(O.permutation_of(piv, 520), perm)


def test_et_zero_pivot_reported():
    A = G.zero_column(300, seed=2, col=77)
    F, piv, info, widths = run_et(A, 64, 16, "always")
    R = A.copy()
    opiv, oinfo = O.getrf(R, "la", schedule=widths, inner=("ll", 16))
    assert info == oinfo == 78 and piv == opiv
    assert np.array_equal(F, R)


def test_et_min_width_is_respected():
    A = G.uniform01(900, seed=4)
    F, piv, info, widths = run_et(A, 128, 16, "signal", min_width=64)
    check_widths(widths, 900, 128, 16)
    j = widths[0]
    for w in widths[1:]:
        assert w >= min(64, 900 - j)
        j += w
    R = A.copy()
    opiv, _ = O.getrf(R, "la", schedule=widths, inner=("ll", 16))
    assert piv == opiv and np.abs(F - R).max() <= 1e-12 * np.abs(R).max()
