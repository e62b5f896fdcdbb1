"""GPU parity: every step of the hot path, called through the C ABI, against the
CPU oracle on the same seeded inputs.

Tolerances (FP64):
  * integer / index work (pivots, interchanges, info codes): bit-exact;
  * inputs whose elimination is exact in binary64 (known-answer, Wilkinson,
    small-integer GEMMs): bit-exact results;
  * general inputs: normwise residual ||P A - L U||_F / ||A||_F <= 1e-13 (the
    FP64 bar), identical pivots, and elementwise
    |F_gpu - F_oracle| <= 1e-12 * max|F_oracle| at these sizes (rounding order
    differs: MFMA accumulation and fused multiply-adds).
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


def dev(A):
    return torch.from_numpy(np.ascontiguousarray(A, dtype=np.float64)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def gpu_getrf(A, variant, nb, nb_inner=0, schedule=None, iters_limit=-1):
    dA = dev(A)
    ipiv, info = mlu.getrf(dA, variant=variant, nb=nb, nb_inner=nb_inner, schedule=schedule,
                           iters_limit=iters_limit)
    F = host(dA)
    k = min(A.shape)
    return F, (host(ipiv)[:k] - 1).tolist(), int(host(info)[0])


def inner_of(nb, nb_inner):
    bi = nb_inner if nb_inner > 0 else min(nb, 16)
    return ("rl", bi)


# ------------------------------------------------------------------ K4: GEMM
@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (37, 53, 19), (128, 128, 16), (300, 257, 64), (513, 129, 256),
                                   (1024, 1024, 256), (130, 700, 33), (64, 4096, 1)])
def test_gemm_update_random(m, n, k):
    rng = np.random.default_rng(m * 7 + n * 3 + k)
    A, B, C = rng.standard_normal((m, k)), rng.standard_normal((k, n)), rng.standard_normal((m, n))
    dC = dev(C)
    mlu.gemm_update(dC, dev(A), dev(B))
    ref = C - A @ B
    bound = 2 * k * np.finfo(float).eps * (np.abs(A) @ np.abs(B) + np.abs(C))
    assert np.all(np.abs(host(dC) - ref) <= bound + 1e-300)


@pytest.mark.parametrize("m,n,k", [(200, 300, 48), (128, 256, 256)])
def test_gemm_update_exact_integers(m, n, k):
    rng = np.random.default_rng(5)
    A = rng.integers(-50, 51, (m, k)).astype(float)
    B = rng.integers(-50, 51, (k, n)).astype(float)
    C = rng.integers(-1000, 1001, (m, n)).astype(float)
    dC = dev(C)
    mlu.gemm_update(dC, dev(A), dev(B))
    assert np.array_equal(host(dC), C - A @ B)


def test_gemm_update_submatrix_strides():
    rng = np.random.default_rng(9)
    big = rng.standard_normal((300, 301))
    d = dev(big)
    # C = big[101:, 37:], A = big[101:, 5:37], B = big[5:37, 37:]  (odd offsets: unaligned path)
    mlu.gemm_update(d[101:, 37:], d[101:, 5:37], d[5:37, 37:])
    ref = big.copy()
    ref[101:, 37:] -= big[101:, 5:37] @ big[5:37, 37:]
    assert np.abs(host(d) - ref).max() <= 1e-13 * np.abs(ref).max()


# ------------------------------------------------------------------ K1: panel kernel
@pytest.mark.parametrize("m", [1, 5, 63, 300, 512, 513, 1024, 1025, 3000, 5000])
@pytest.mark.parametrize("bw", [1, 7, 8, 9, 16])
def test_panel_block_uniform(m, bw):
    if bw > m:
        pytest.skip("bw > m")
    A = G.uniform01(m, bw, seed=m + bw)
    dA = dev(A)
    ipiv, info = mlu.getf2_block(dA)
    F = host(dA)
    piv = (host(ipiv)[:bw] - 1).tolist()
    R = A.copy()
    opiv = O.lu_unb(R)
    assert int(host(info)[0]) == 0
    assert piv == opiv
    assert np.abs(F - R).max() <= 1e-13 * max(1.0, np.abs(R).max())


@pytest.mark.parametrize("m,bw", [(40, 16), (2000, 16), (1500, 16), (4100, 8), (17000, 16)])
def test_panel_block_known_answer_exact(m, bw):
    A, perm, L, U = G.known_answer(m, bw, seed=m)
    dA = dev(A)
    ipiv, info = mlu.getf2_block(dA)
    F = host(dA)
    piv = (host(ipiv)[:bw] - 1).tolist()
    R = A.copy()
    opiv = O.lu_unb(R)
    assert piv == opiv
    assert np.array_equal(F, R)


def test_panel_block_ties_and_zero_pivot():
    W = G.wilkinson_growth(16)
    dW = dev(W)
    ipiv, info = mlu.getf2_block(dW)
    assert (host(ipiv)[:16] - 1).tolist() == list(range(16))
    R = W.copy()
    O.lu_unb(R)
    assert np.array_equal(host(dW), R)
    # an all-zero first column: info = 1, no division, factorization continues
    Z = G.uniform01(700, 8, seed=3)
    Z[:, 0] = 0.0
    dZ = dev(Z)
    ipiv, info = mlu.getf2_block(dZ)
    R = Z.copy()
    inf_ = [0]
    opiv = O.lu_unb(R, info=inf_)
    assert int(host(info)[0]) == 1 == inf_[0]
    assert (host(ipiv)[:8] - 1).tolist() == opiv
    assert np.abs(host(dZ) - R).max() <= 1e-13


@pytest.mark.parametrize("m,bw,fail_at", [(3000, 16, None), (3000, 16, 0), (3000, 16, 6), (5000, 8, 7), (300, 16, None), (300, 16, 9),
                                           (1000, 16, None), (17000, 16, 11)])
def test_panel_block_speculation_paths(m, bw, fail_at):
    # Tall blocks are first factored speculatively with pivots from the first
    # 512 rows; pivot rows placed below them make that guess fail at column
    # `fail_at` and the block is redone exactly.  Every path must give the
    # partial-pivoting factorization, bit for bit on this exact input.
    perm = G.leader_perm(m, bw, 64, fail_at, seed=m + bw)
    A, perm, L, U = G.known_answer(m, bw, seed=m, perm=perm)
    dA = dev(A)
    ipiv, info = mlu.getf2_block(dA)
    F = host(dA)
    piv = (host(ipiv)[:bw] - 1).tolist()
    R = A.copy()
    opiv = O.lu_unb(R)
    assert int(host(info)[0]) == 0
    assert piv == opiv
    assert np.array_equal(F, R)
    assert np.array_equal(O.permutation_of(piv, m)[:bw], perm[:bw])


# ------------------------------------------------------------------ K2: interchanges
@pytest.mark.parametrize("m,ncols,k1,k2", [(50, 7, 0, 10), (1000, 300, 100, 356), (600, 1000, 0, 300),
                                           (64, 33, 60, 64)])
def test_laswp_random_interchanges(m, ncols, k1, k2):
    rng = np.random.default_rng(m + ncols)
    A = rng.standard_normal((m, ncols))
    piv = np.arange(m, dtype=np.int64)
    for c in range(k1, k2):
        r = rng.random()
        if r < 0.2:
            piv[c] = c
        elif r < 0.5 and c > k1:
            q = rng.integers(k1, c)          # reuse an earlier far row when still legal
            piv[c] = piv[q] if piv[q] >= c else rng.integers(c, m)
        else:
            piv[c] = rng.integers(c, m)
    d_ipiv = torch.from_numpy((piv + 1).astype(np.int32)).to(DEV)
    dA = dev(A)
    info = torch.zeros(1, dtype=torch.int32, device=DEV)
    mlu.laswp(dA, k1, k2, d_ipiv, info)
    R = A.copy()
    for c in range(k1, k2):
        p = int(piv[c])
        R[[c, p], :] = R[[p, c], :]
    assert int(host(info)[0]) == 0
    assert np.array_equal(host(dA), R)


def test_laswp_rejects_bad_index():
    A = np.arange(40.0).reshape(10, 4)
    d_ipiv = torch.tensor([3, 1, 11], dtype=torch.int32, device=DEV)   # step 1 -> row 0 (< 1), step 2 -> 10 (>= m)
    info = torch.zeros(1, dtype=torch.int32, device=DEV)
    dA = dev(A)
    mlu.laswp(dA, 0, 3, d_ipiv, info)
    assert int(host(info)[0]) == mlu.MLU_INFO_BAD_PIVOT
    R = A.copy()
    R[[0, 2], :] = R[[2, 0], :]
    assert np.array_equal(host(dA), R)


# ------------------------------------------------------------------ K3: triangular solves
@pytest.mark.parametrize("uplo", ["L", "U"])
@pytest.mark.parametrize("diag", ["U", "N"])
@pytest.mark.parametrize("n,k", [(12, 5), (40, 100), (100, 3), (256, 300)])
def test_trsm_exact_known_solution(uplo, diag, n, k):
    rng = np.random.default_rng(n + k)
    T = rng.integers(-7, 8, (n, n)) / 8.0
    T[np.arange(n), np.arange(n)] = 2.0 ** rng.integers(-1, 2, n) * rng.choice([-1, 1], n)
    Tt = np.tril(T) if uplo == "L" else np.triu(T)
    if diag == "U":
        Tt = Tt.copy()
        Tt[np.arange(n), np.arange(n)] = 1.0
    X = rng.integers(-3, 4, (n, k)).astype(float)
    B = Tt @ X
    if np.abs(B).max() > 2.0 ** 40:
        pytest.skip("values too large to stay exact")
    dB = dev(B)
    mlu.trsm(dev(T), dB, uplo, diag)
    Y = O.trsm(T, B, uplo, diag)
    assert np.array_equal(Y, X)
    assert np.array_equal(host(dB), X)


@pytest.mark.parametrize("uplo", ["L", "U"])
def test_trsm_config0_operand(uplo):
    T = G.tri_operand(256, seed=0)
    if uplo == "U":
        T = np.ascontiguousarray(T.T)
    B = np.random.default_rng(2).standard_normal((256, 64))
    dB = dev(B)
    mlu.trsm(dev(T), dB, uplo, "N")
    X = host(dB)
    Tt = np.tril(T) if uplo == "L" else np.triu(T)
    inf = lambda M: np.abs(M).sum(axis=1).max()
    assert inf(Tt @ X - B) / (inf(Tt) * inf(X)) < 256 * np.finfo(float).eps
    # the solution grows to ~1e200 (off-diagonal ~16 over a diagonal in [1, 2]),
    # so only the backward error is meaningful for this operand


@pytest.mark.parametrize("uplo", ["L", "U"])
@pytest.mark.parametrize("diag", ["U", "N"])
def test_trsm_well_conditioned_elementwise(uplo, diag):
    rng = np.random.default_rng(8)
    n = 300
    T = rng.standard_normal((n, n)) / n
    T[np.arange(n), np.arange(n)] = 1.0 + rng.random(n)
    B = rng.standard_normal((n, 77))
    dB = dev(B)
    mlu.trsm(dev(T), dB, uplo, diag)
    Y = O.trsm(T, B, uplo, diag)
    assert np.abs(host(dB) - Y).max() <= 1e-13 * np.abs(Y).max()


# ------------------------------------------------------------------ whole path: config 0
CONFIG0 = [(v, nb, nbi) for v in ("rl", "ll", "la") for nb, nbi in ((1, 0), (32, 0), (32, 8))]


@pytest.mark.parametrize("variant,nb,nb_inner", CONFIG0)
@pytest.mark.parametrize("recipe", ["spd", "uniform"])
def test_getrf_config0(variant, nb, nb_inner, recipe):
    n = 256
    A = G.spd_bbt(n, seed=0) if recipe == "spd" else G.uniform01(n, seed=0)
    F, piv, info = gpu_getrf(A, variant, nb, nb_inner)
    R = A.copy()
    opiv, oinfo = O.getrf(R, variant, nb=nb, inner=inner_of(nb, nb_inner))
    assert info == oinfo == 0
    assert piv == opiv
    assert np.abs(F - R).max() <= 1e-12 * np.abs(R).max()
    pc = I.postcondition(A, F, piv)
    assert pc["rel_frob"] <= 1e-13 and pc["l_max"] <= 1.0


@pytest.mark.parametrize("seed", [1, 2])
def test_getrf_config0_other_seeds(seed):
    A = G.spd_bbt(256, seed=seed)
    for v in ("rl", "ll", "la"):
        F, piv, info = gpu_getrf(A, v, 32)
        assert info == 0 and piv == list(range(256))
        assert I.postcondition(A, F, piv)["rel_frob"] <= 1e-13


@pytest.mark.parametrize("variant", ["rl", "ll", "la"])
@pytest.mark.parametrize("shape,nb", [((64, 64), 8), ((200, 150), 32), ((150, 200), 32), ((1, 1), 4),
                                      ((513, 40), 16), ((40, 513), 16), ((300, 300), 1), ((257, 257), 300)])
def test_getrf_known_answer_exact(variant, shape, nb):
    m, n = shape
    A, perm, L, U = G.known_answer(m, n, seed=m * 7 + n)
    F, piv, info = gpu_getrf(A, variant, nb)
    R = A.copy()
    opiv, _ = O.getrf(R, variant, nb=nb, inner=inner_of(nb, 0))
    assert info == 0 and piv == opiv
    assert np.array_equal(F, R)
    k = min(m, n)
    got = O.permutation_of(piv, m)
    assert np.array_equal(got[:k], perm[:k])


@pytest.mark.parametrize("variant", ["rl", "ll", "la"])
def test_getrf_wilkinson_exact(variant):
    W = G.wilkinson_growth(53)
    F, piv, info = gpu_getrf(W, variant, 8, 4)
    assert piv == list(range(53))
    assert np.array_equal(np.triu(F)[:, -1], 2.0 ** np.arange(53))


@pytest.mark.parametrize("variant", ["rl", "ll", "la"])
def test_getrf_zero_pivot(variant):
    for col in (0, 17, 40):
        A = G.zero_column(48, seed=4, col=col)
        F, piv, info = gpu_getrf(A, variant, 16, 8)
        R = A.copy()
        opiv, oinfo = O.getrf(R, variant, nb=16, inner=("rl", 8))
        assert info == oinfo == col + 1
        assert piv == opiv and np.array_equal(F, R)


@pytest.mark.parametrize("variant", ["rl", "ll", "la"])
def test_getrf_random_schedules(variant):
    A = G.uniform01(180, seed=11)
    for t in range(3):
        sched = G.random_schedule(180, seed=t, max_b=40)
        F, piv, info = gpu_getrf(A, variant, 8, 0, schedule=sched)
        R = A.copy()
        opiv, _ = O.getrf(R, variant, schedule=sched, inner=("rl", 8))
        assert piv == opiv
        assert np.abs(F - R).max() <= 1e-12 * np.abs(R).max()


@pytest.mark.parametrize("variant", ["rl", "ll", "la"])
def test_getrf_loop_invariant_after_each_iteration(variant):
    n, nb = 96, 16
    A = G.uniform01(n, seed=12)
    sched = O.schedule_from(n, nb)
    for s in range(len(sched) + 1):
        F, piv, info = gpu_getrf(A, variant, nb, 8, iters_limit=s)
        j = sum(sched[:s])
        if variant == "rl":
            err = I.check_rl(A, F, piv[:j], j)
        elif variant == "ll":
            err = I.check_ll(A, F, piv[:j], j, lazy=True)
        else:
            bp = sched[s] if s < len(sched) else 0
            err = I.check_la(A, F, piv[:j], [p - j for p in piv[j:j + bp]], j, bp)
        assert err < 1e-14, (variant, s, err)
        R = A.copy()
        opiv, _ = O.getrf(R, variant, nb=nb, inner=("rl", 8), iters_limit=s)
        assert np.abs(F - R).max() <= 1e-12 * np.abs(R).max()


def test_getrf_variants_agree_moderate_n():
    A = G.uniform01(1000, seed=13)
    res = {}
    for v in ("rl", "ll", "la"):
        res[v] = gpu_getrf(A, v, 128)
        assert I.postcondition(A, res[v][0], res[v][1])["rel_frob"] <= 1e-13
    assert res["rl"][1] == res["ll"][1] == res["la"][1]
    for v in ("ll", "la"):
        assert np.abs(res[v][0] - res["rl"][0]).max() <= 1e-11 * np.abs(res["rl"][0]).max()


@pytest.mark.parametrize("variant", ["rl", "la"])
def test_getrf_spd_moderate_n(variant):
    # tall panels with no interchange: the speculative panel path is kept
    A = G.spd_bbt(1500, seed=3)
    F, piv, info = gpu_getrf(A, variant, 256, 16)
    R = A.copy()
    opiv, _ = O.getrf(R, "rl", nb=256, inner=("rl", 16))
    assert info == 0 and piv == opiv == list(range(1500))
    assert np.abs(F - R).max() <= 1e-12 * np.abs(R).max()


def test_getrs_solves():
    A, perm, L, U = G.known_answer(64, 64, seed=21)
    x = np.random.default_rng(4).integers(-5, 6, (64, 3)).astype(float)
    b = A @ x
    dA = dev(A)
    ipiv, info = mlu.getrf(dA, "rl", nb=16)
    db = dev(b)
    mlu.getrs(dA, ipiv, db)
    assert np.array_equal(host(db), x)
    A2 = G.uniform01(300, seed=5)
    b2 = np.random.default_rng(6).standard_normal((300, 4))
    dA = dev(A2)
    ipiv, info = mlu.getrf(dA, "la", nb=64)
    db = dev(b2)
    mlu.getrs(dA, ipiv, db)
    X = host(db)
    R = A2.copy()
    opiv, _ = O.getrf(R, "rl", nb=64)
    Xo = O.getrs(R, opiv, b2)
    assert np.abs(X - Xo).max() <= 1e-11 * np.abs(Xo).max()


def test_empty_and_degenerate_shapes():
    for (m, n) in ((0, 5), (5, 0), (0, 0)):
        dA = torch.zeros((max(m, 1), max(n, 1)), dtype=torch.float64, device=DEV)[:m, :n]
        if m == 0 or n == 0:
            info = torch.full((1,), 7, dtype=torch.int32, device=DEV)
            ipiv = torch.zeros(1, dtype=torch.int32, device=DEV)
            work = mlu.workspace(DEV)
            rc = mlu.mlu_dgetrf(mlu._stream(), m, n, dA.data_ptr() if dA.numel() else 1, max(n, 1),
                                ipiv.data_ptr(), info.data_ptr(), 0, 4, 0, 0, None, 0, -1, work.data_ptr(),
                                work.numel())
            assert rc == 0
            assert int(host(info)[0]) == 0
