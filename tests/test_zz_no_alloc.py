"""The entry point that allocates nothing (mlu_dgetrf_noalloc): through the C
ABI, its results against mlu_dgetrf with a caller workspace on the same
inputs, on two calls in a row, the second on a smaller matrix (the shared
scratch array keeps the first call's contents, so the second shows that each
call clears what must start at zero).  Index work bit-exact, factors
bit-equal (the same kernels in the same order)."""
import numpy as np
import pytest
import torch

import inputs as G
from paper_1611_06365_amd import mlu

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    mlu.load()
    assert mlu.mlu_init() == 0
    yield
    torch.cuda.synchronize()


def run_both(A, variant, nb, nb_inner=0, inner="rl"):
    m, n = A.shape
    k = min(m, n)
    v = mlu.VARIANT_IDS[variant]
    iv = mlu.VARIANT_IDS[inner]
    ref = torch.from_numpy(A.copy()).to(DEV)
    ipiv_r = torch.zeros(max(k, 1), dtype=torch.int32, device=DEV)
    info_r = torch.full((1,), -7, dtype=torch.int32, device=DEV)
    work = mlu.workspace(DEV)
    s = mlu._stream()
    rc = mlu.mlu_dgetrf(s, m, n, ref.data_ptr(), n, ipiv_r.data_ptr(), info_r.data_ptr(), v, nb, nb_inner, iv,
                        None, 0, -1, work.data_ptr(), work.numel())
    assert rc == 0
    got = torch.from_numpy(A.copy()).to(DEV)
    ipiv_g = torch.zeros(max(k, 1), dtype=torch.int32, device=DEV)
    info_g = torch.full((1,), -7, dtype=torch.int32, device=DEV)
    rc = mlu.mlu_dgetrf_noalloc(s, m, n, got.data_ptr(), n, ipiv_g.data_ptr(), info_g.data_ptr(), v, nb, nb_inner,
                                iv, None, 0, -1)
    assert rc == 0
    torch.cuda.synchronize()
    assert int(info_g.item()) == int(info_r.item()) == 0
    assert torch.equal(ipiv_g[:k], ipiv_r[:k])
    assert torch.equal(got, ref)
    return got


@pytest.mark.parametrize("variant,nb", [("la", 128), ("rl", 64), ("ll", 96)])
def test_noalloc_matches_workspace_entry_two_calls(variant, nb):
    big = G.uniform01(1500, 1400, seed=31)
    small = G.uniform01(333, 300, seed=32)
    run_both(big, variant, nb)
    run_both(small, variant, nb)


def test_noalloc_rejects_tall_matrices_before_any_work():
    rc = mlu.mlu_dgetrf_noalloc(mlu._stream(), 33281, 4, 1024, 4, 2048, 4096, 2, 64, 0, 0, None, 0, -1)
    assert rc == -2
