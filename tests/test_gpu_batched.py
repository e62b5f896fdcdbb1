"""GPU parity of the batched LU (mlu_dgetrf_batched / mlu_sgetrf_batched):
every matrix of a mixed-size batch against the oracle, on the same inputs.

Bars (FP64): pivots identical, factors within 1e-12 * max|F_oracle| (orders up
to 300; rounding order differs), residual ||P A - L U||_F / ||A||_F <= 1e-13;
known-answer matrices bit-exact; info codes exact.  FP32: residual
<= 1e-5 (about 64 n u_32 at these orders) and legal pivots (|L| <= 1).
Graph capture: replays of a captured call reproduce the eager result bit for
bit, with eager work and synchronizations between the replays.
"""
import numpy as np
import pytest
import torch

import inputs as G
import oracle as O
from oracle import invariants as I
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


SIZES = [1, 2, 3, 7, 16, 31, 32, 33, 47, 63, 64, 65, 96, 100, 127, 128, 129, 160, 200, 255, 256, 257, 300]


def make_batch(seed=0):
    rng = np.random.default_rng(seed)
    mats = []
    for i, n in enumerate(SIZES + list(rng.integers(1, 150, 40))):
        n = int(n)
        mats.append(G.uniform01(n, seed=100 + i) if i % 3 else G.spd_bbt(n, seed=100 + i))
    return mats


@pytest.mark.parametrize("nb", [16, 32])
def test_batched_fp64_against_oracle(nb):
    mats = make_batch()
    dmats = [torch.from_numpy(a.copy()).to(DEV) for a in mats]
    plan = mlu.getrf_batched(dmats, nb=nb)
    info = host(plan.info)
    for i, (a, d) in enumerate(zip(mats, dmats)):
        n = a.shape[0]
        F = host(d)
        piv = (host(plan.pivots(i)) - 1).tolist()
        R = a.copy()
        opiv, oinfo = O.getrf(R, "rl", nb=32)
        assert info[i] == oinfo == 0, i
        assert piv == opiv, (i, n)
        assert np.abs(F - R).max() <= 1e-12 * max(1.0, np.abs(R).max()), (i, n)
        assert I.postcondition(a, F, piv)["rel_frob"] <= 1e-13, (i, n)


def _planted(n, seed, row, col, value=1.0e6):
    """A = B B^T + n I (diagonal pivots throughout) with one entry planted
    below the diagonal, which makes row `row` the pivot of column `col`."""
    a = G.spd_bbt(n, seed=seed)
    a[row, col] = value
    return a


@pytest.mark.parametrize("nb", [16, 32])
def test_batched_diagonal_speculation_and_its_misses(nb):
    """Diagonal pivots are tried first on every panel: matrices whose pivots
    stay on the diagonal, and matrices where the guess fails in the first
    panel (in the wave holding the pivot rows or in another one) or only in a
    later panel (the rest of the matrix then goes column by column), all
    against the oracle."""
    mats = [G.spd_bbt(n, seed=300 + n) for n in (5, 40, 100, 300, 500)]
    mats += [_planted(100, 1, 10, 3), _planted(500, 2, 400, 5), _planted(300, 3, 150, 40),
             _planted(500, 4, 480, 100), _planted(200, 5, 199, 198)]
    dmats = [torch.from_numpy(a.copy()).to(DEV) for a in mats]
    plan = mlu.getrf_batched(dmats, nb=nb)
    info = host(plan.info)
    for i, (a, d) in enumerate(zip(mats, dmats)):
        n = a.shape[0]
        F = host(d)
        piv = (host(plan.pivots(i)) - 1).tolist()
        R = a.copy()
        opiv, oinfo = O.getrf(R, "rl", nb=32)
        assert info[i] == oinfo == 0, i
        assert piv == opiv, (i, n)
        assert np.abs(F - R).max() <= 1e-12 * max(1.0, np.abs(R).max()), (i, n)
        assert I.postcondition(a, F, piv)["rel_frob"] <= 1e-13, (i, n)
    # the planted rows are the pivots of their columns, the others stay put
    assert (host(plan.pivots(5)) - 1)[3] == 10
    assert (host(plan.pivots(7)) - 1)[40] == 150
    assert all((host(plan.pivots(k)) - 1).tolist() == list(range(mats[k].shape[0])) for k in range(5))


@pytest.mark.parametrize("top,max_n", [(128, None), (200, None), (256, 512), (100, 200)])
def test_batched_size_classes(top, max_n):
    """Batches whose largest order (or stated max_n) leaves some of the three
    size classes (orders above 256, above 128, the rest) empty or not
    launched, orders at the class edges included, against the oracle."""
    rng = np.random.default_rng(top)
    ns = [n for n in (1, 64, 127, 128, 129, 200, 255, 256) if n <= top] + list(rng.integers(1, top + 1, 20))
    mats = [G.uniform01(int(n), seed=500 + i) for i, n in enumerate(ns)]
    dmats = [torch.from_numpy(a.copy()).to(DEV) for a in mats]
    plan = mlu.BatchPlan(dmats, max_n=max_n, nb=32)
    plan.run()
    info = host(plan.info)
    for i, (a, d) in enumerate(zip(mats, dmats)):
        F = host(d)
        piv = (host(plan.pivots(i)) - 1).tolist()
        R = a.copy()
        opiv, oinfo = O.getrf(R, "rl", nb=32)
        assert info[i] == oinfo == 0, i
        assert piv == opiv, (i, a.shape[0])
        assert np.abs(F - R).max() <= 1e-12 * max(1.0, np.abs(R).max()), (i, a.shape[0])


@pytest.mark.parametrize("nb", [0, 32])
def test_batched_known_answer_and_zero_pivot(nb):
    mats, expect = [], []
    for i, n in enumerate([5, 33, 64, 97, 130]):
        A, perm, L, U = G.known_answer(n, n, seed=7 + i)
        mats.append(A)
        expect.append(0)
    for col in (0, 17, 40):
        mats.append(G.zero_column(48, seed=4, col=col))
        expect.append(col + 1)
    dmats = [torch.from_numpy(a.copy()).to(DEV) for a in mats]
    plan = mlu.getrf_batched(dmats, nb=nb)
    info = host(plan.info)
    for i, (a, d) in enumerate(zip(mats, dmats)):
        R = a.copy()
        opiv, oinfo = O.getrf(R, "rl", nb=32)
        assert info[i] == oinfo == expect[i]
        assert (host(plan.pivots(i)) - 1).tolist() == opiv
        assert np.array_equal(host(d), R), i


def test_batched_invalid_entries_are_reported_and_untouched():
    ok = torch.from_numpy(G.uniform01(40, seed=1)).to(DEV)
    big = torch.from_numpy(G.uniform01(70, seed=2)).to(DEV)
    big0 = big.clone()
    empty = torch.zeros((0, 0), dtype=torch.float64, device=DEV)
    plan = mlu.BatchPlan([ok, big, empty], max_n=64)   # 70 > max_n
    plan.run()
    info = host(plan.info)
    assert info.tolist() == [0, -1, 0]
    assert torch.equal(big, big0)


@pytest.mark.parametrize("nb", [16, 32])
def test_batched_fp32(nb):
    mats = make_batch(seed=3)[:40]
    dmats = [torch.from_numpy(a.astype(np.float32)).to(DEV) for a in mats]
    plan = mlu.getrf_batched(dmats, nb=nb)
    info = host(plan.info)
    for i, (a, d) in enumerate(zip(mats, dmats)):
        a32 = a.astype(np.float32).astype(np.float64)
        F = host(d).astype(np.float64)
        piv = (host(plan.pivots(i)) - 1).tolist()
        assert info[i] == 0
        res = I.postcondition(a32, F, piv)["rel_frob"]
        assert res <= 1e-5, (i, a.shape[0], res)
        assert np.abs(np.tril(F, -1)).max() <= 1.0


def test_batched_graph_replays_match_eager():
    mats = make_batch(seed=5)[:30]
    pristine = [torch.from_numpy(a.copy()).to(DEV) for a in mats]
    work = [p.clone() for p in pristine]
    plan = mlu.BatchPlan(work)
    plan.run()                      # eager reference (also raises the LDS limit outside capture)
    ref = [w.clone() for w in work]
    ref_piv = plan.ipiv.clone()
    for w, p in zip(work, pristine):
        w.copy_(p)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            plan.run(stream=s)
    for rep in range(3):
        for w, p in zip(work, pristine):
            w.copy_(p)
        torch.cuda.synchronize()
        _ = (torch.ones(1000, device=DEV) * rep).sum().item()   # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(plan.ipiv, ref_piv), rep
        for w, r in zip(work, ref):
            assert torch.equal(w, r), rep


def _bench_batch(dt, count=20000):
    """The bench's batched workload: orders n ~ U{8..512} (seed 0), each
    A = B B^T + n I with B ~ N(0, 1) drawn on the device per order (seed 1)."""
    rng = np.random.default_rng(0)
    ns = rng.integers(8, 513, count)
    offs = np.concatenate([[0], np.cumsum(ns.astype(np.int64) ** 2)])
    buf = torch.empty(int(offs[-1]), dtype=dt, device=DEV)
    g = torch.Generator(device=DEV)
    g.manual_seed(1)
    for n in np.unique(ns):
        idx = np.nonzero(ns == n)[0]
        b = torch.randn(len(idx), int(n), int(n), generator=g, dtype=torch.float64, device=DEV)
        a = torch.bmm(b, b.transpose(1, 2).contiguous())
        a.diagonal(dim1=1, dim2=2).add_(float(n))
        for t, i in enumerate(idx):
            buf[int(offs[i]):int(offs[i + 1])].copy_(a[t].reshape(-1))
        del a, b
    mats = [buf[int(offs[i]):int(offs[i + 1])].view(int(n), int(n)) for i, n in enumerate(ns)]
    return ns, buf, mats


@pytest.mark.parametrize("dt,nb", [(torch.float64, 16), (torch.float64, 32), (torch.float32, 32)])
def test_batched_full_bench_configuration(dt, nb):
    """The full 20 000-matrix launch the bench times: every info code, and 120
    sampled matrices (the largest and smallest orders included) against the
    oracle (FP64: pivots identical, factors within 1e-12 * max|F|) or by
    residual and legal pivots (FP32)."""
    ns, buf, mats = _bench_batch(dt)
    rng = np.random.default_rng(7)
    pick = sorted(set(rng.choice(len(ns), 118, replace=False).tolist()) | {int(ns.argmax()), int(ns.argmin())})
    before = {i: mats[i].double().cpu().numpy() for i in pick}
    plan = mlu.BatchPlan(mats, max_n=512, nb=nb)
    plan.run()
    info = host(plan.info)
    assert (info == 0).all()
    for i in pick:
        a = before[i]
        F = host(mats[i]).astype(np.float64)
        piv = (host(plan.pivots(i)) - 1).tolist()
        if dt == torch.float64:
            R = a.copy()
            opiv, oinfo = O.getrf(R, "rl", nb=32)
            assert piv == opiv, (i, a.shape[0])
            assert np.abs(F - R).max() <= 1e-12 * np.abs(R).max(), (i, a.shape[0])
        else:
            assert I.postcondition(a, F, piv)["rel_frob"] <= 1e-5, (i, a.shape[0])
            assert np.abs(np.tril(F, -1)).max() <= 1.0
    del plan, mats, buf
    torch.cuda.empty_cache()
