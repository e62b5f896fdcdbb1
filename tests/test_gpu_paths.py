"""GPU parity of launch paths the other parity files do not reach.

  * the panel factorization's inner variant (Section 4.2, outer / inner LU:
    right-looking or left-looking inside the panel) and the inner block size
    b_i = 32 (a 32-column diagonal block in two register passes), against the
    oracle run with the same inner variant and b_i: identical pivots, factors
    within 1e-12 * max|F_oracle| (rounding order differs), bit-exact on
    known-answer inputs whose elimination is exact in binary64;
  * the trailing update on the 128 x 128 tile (at least 128 tiles, with ragged
    edges in both dimensions), exact on integers and within the rounding bound
    on random inputs;
  * n = 3001 (a ragged last block) with nb = 32 and 64 against the C oracle;
  * look-ahead at orders that are not multiples of the 128 x 128 tile, odd
    leading dimensions among them: residual, |L| <= 1, legal interchanges;
  * look-ahead with early termination at n = 16384 for every stop mode:
    normwise residual <= 1e-13, |L| <= 1, legal interchanges, realized widths
    that cover the matrix;
  * look-ahead without worker sharing bit-identical to look-ahead;
  * one look-ahead call captured in a stream graph (its library stream forked
    and joined with events), replayed several times with other work and
    synchronizations between the replays: every replay bit-equal to the eager
    call;
  * plain LU-IR stopping once its corrections diverge (BF16 products at
    kappa = 1e5) instead of running every allowed correction.
"""
import numpy as np
import pytest
import torch

import inputs as G
import inputs.device as D
import oracle as O
from oracle import c_oracle
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


def gpu_getrf(A, variant, nb, nb_inner, inner):
    dA = dev(A)
    ipiv, info = mlu.getrf(dA, variant=variant, nb=nb, nb_inner=nb_inner, inner=inner)
    k = min(A.shape)
    return host(dA), (host(ipiv)[:k] - 1).tolist(), int(host(info)[0])


# ------------------------------------------------------------ inner variant, b_i
@pytest.mark.parametrize("variant", ["rl", "ll", "la"])
@pytest.mark.parametrize("inner", ["rl", "ll"])
@pytest.mark.parametrize("shape,nb,bi", [((300, 300), 64, 32), ((333, 270), 100, 24), ((270, 333), 64, 16),
                                         ((600, 600), 96, 32), ((1100, 700), 256, 32)])
def test_inner_variant_and_block_against_oracle(variant, inner, shape, nb, bi):
    m, n = shape
    A = G.uniform01(m, n, seed=m + 3 * n + bi)
    F, piv, info = gpu_getrf(A, variant, nb, bi, inner)
    R = A.copy()
    opiv, oinfo = O.getrf(R, variant, nb=nb, inner=(inner, bi))
    assert info == oinfo == 0
    assert piv == opiv
    err = np.abs(F - R).max() / np.abs(R).max()
    print(f"{variant} inner={inner} b_i={bi} {m}x{n} nb={nb}: max|F - oracle| / max|oracle| = {err:.2e}",
          flush=True)
    assert err <= 1e-12


@pytest.mark.parametrize("variant", ["rl", "la", "ll"])
@pytest.mark.parametrize("inner,bi", [("rl", 32), ("ll", 32), ("ll", 16), ("rl", 20)])
def test_inner_variant_known_answer_exact(variant, inner, bi):
    m = n = 160
    A, perm, L, U = G.known_answer(m, n, seed=bi + len(inner))
    F, piv, info = gpu_getrf(A, variant, 64, bi, inner)
    R = A.copy()
    opiv, oinfo = O.getrf(R, variant, nb=64, inner=(inner, bi))
    assert info == oinfo == 0
    assert piv == opiv
    assert np.array_equal(F, R)


def test_inner_ll_iters_limit_states_match_oracle():
    A = G.uniform01(200, seed=17)
    for s in (1, 2, 4):
        dA = dev(A)
        ipiv, info = mlu.getrf(dA, variant="rl", nb=48, nb_inner=32, inner="ll", iters_limit=s)
        F = host(dA)
        R = A.copy()
        opiv, _ = O.getrf(R, "rl", nb=48, inner=("ll", 32), iters_limit=s)
        j = len(opiv)
        assert (host(ipiv)[:j] - 1).tolist() == opiv
        assert np.abs(F - R).max() <= 1e-12 * np.abs(R).max()


# ------------------------------------------------------------ 128 x 128 tiles
@pytest.mark.parametrize("m,n,k", [(2000, 1900, 256), (1537, 2049, 48)])
def test_gemm_big_tile_ragged_random(m, n, k):
    assert ((m + 127) // 128) * ((n + 127) // 128) >= 128   # the 128 x 128 tile path
    rng = np.random.default_rng(m + n + k)
    A, B, C = rng.standard_normal((m, k)), rng.standard_normal((k, n)), rng.standard_normal((m, n))
    dC = dev(C)
    mlu.gemm_update(dC, dev(A), dev(B))
    ref = C - A @ B
    bound = 2 * k * np.finfo(float).eps * (np.abs(A) @ np.abs(B) + np.abs(C))
    assert np.all(np.abs(host(dC) - ref) <= bound + 1e-300)


def test_gemm_big_tile_ragged_exact_integers_and_offsets():
    m, n, k = 2000, 1900, 256
    rng = np.random.default_rng(11)
    big = rng.integers(-40, 41, (m + k + 3, n + k + 5)).astype(float)
    d = dev(big)
    # C, A, B inside one matrix at odd offsets (the unaligned staging path)
    C0, A0, B0 = (k + 3, k + 5), (k + 3, 3), (3, k + 5)
    ref = big.copy()
    ref[C0[0]:C0[0] + m, C0[1]:C0[1] + n] -= (big[A0[0]:A0[0] + m, A0[1]:A0[1] + k]
                                             @ big[B0[0]:B0[0] + k, B0[1]:B0[1] + n])
    mlu.gemm_update(d[C0[0]:C0[0] + m, C0[1]:C0[1] + n], d[A0[0]:A0[0] + m, A0[1]:A0[1] + k],
                    d[B0[0]:B0[0] + k, B0[1]:B0[1] + n])
    assert np.array_equal(host(d), ref)
    # aligned operands (the vector staging path)
    A = rng.integers(-40, 41, (m, k)).astype(float)
    B = rng.integers(-40, 41, (k, n)).astype(float)
    C = rng.integers(-1000, 1001, (m, n)).astype(float)
    dC = dev(C)
    mlu.gemm_update(dC, dev(A), dev(B))
    assert np.array_equal(host(dC), C - A @ B)


# ------------------------------------------------------------ n = 3001 vs the C oracle
_c = {}


@pytest.mark.parametrize("recipe", ["spd", "uniform"])
@pytest.mark.parametrize("variant,nb,bi", [("rl", 32, 16), ("la", 64, 16), ("ll", 64, 16), ("la", 64, 32),
                                           ("rl", 64, 32)])
def test_n3001_against_c_oracle(recipe, variant, nb, bi):
    n = 3001
    A = G.spd_bbt(n, seed=1) if recipe == "spd" else G.uniform01(n, seed=1)
    if recipe not in _c:
        R = np.ascontiguousarray(A.copy())
        opiv, oinfo = c_oracle.dgetrf_rl(R, nb=64)
        _c[recipe] = (R, opiv, oinfo)
    R, opiv, oinfo = _c[recipe]
    F, piv, info = gpu_getrf(A, variant, nb, bi, "rl")
    assert info == oinfo == 0
    assert np.array_equal(np.asarray(piv) + 1, opiv)
    err = float(np.abs(F - R).max() / np.abs(R).max())
    nerr = float(np.linalg.norm(F - R) / np.linalg.norm(R))
    print(f"{recipe} n=3001 {variant} nb={nb} b_i={bi}: max rel {err:.2e}, normwise {nerr:.2e}", flush=True)
    if recipe == "spd":
        assert err <= 1e-12
    else:
        assert nerr <= 1e-12 and err <= 1e-10


# ------------------------------------------------------------ ET at full size
def perm_of(ipiv1):
    piv = ipiv1.astype(np.int64) - 1
    perm = np.arange(piv.size)
    for c, p in enumerate(piv):
        perm[c], perm[p] = perm[p], perm[c]
    return perm


def properties(A, F, ipiv):
    n = A.shape[0]
    ip = ipiv.cpu().numpy()
    assert ip.min() >= 1 and ip.max() <= n
    assert np.all(ip >= np.arange(1, n + 1)), "an interchange picked a row above the diagonal"
    L = torch.tril(F, -1)
    lmax = float(L.abs().max())
    L.diagonal().fill_(1.0)
    LU = L @ torch.triu(F)
    del L
    PA = A[torch.from_numpy(perm_of(ip)).to(A.device)]
    res = float(torch.linalg.norm(PA - LU) / torch.linalg.norm(A))
    return res, lmax


@pytest.mark.parametrize("force", ["never", "always", "signal"])
def test_et_fullsize(force):
    n, nb = 16384, 256
    A = D.spd_bbt(n, seed=0, device=DEV)
    F = A.clone()
    ipiv, info, widths = mlu.getrf_et(F, nb=nb, nb_inner=16, force=force)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    assert sum(widths) == n and widths[0] == nb and all(1 <= w <= nb for w in widths)
    if force == "never":
        assert widths == [nb] * (n // nb)
    if force == "always":
        assert all(w == 16 for w in widths[1:])
    res, lmax = properties(A, F, ipiv)
    print(f"et n={n} nb={nb} force={force}: {len(widths)} panels, residual {res:.2e}, max|L| {lmax:.3f}",
          flush=True)
    assert res <= 1e-13 and lmax <= 1.0
    del F, A
    torch.cuda.empty_cache()


# ------------------------------------------------------------ LA at orders off the tile grid
@pytest.mark.parametrize("n,recipe", [(8191, "uniform"), (9000, "spd"), (12289, "spd"), (12289, "uniform")])
def test_la_orders_off_the_tile_grid(n, recipe):
    """RU2 over the whole 128 x 128 tiles with the partial last tile row and
    column after them (orders that are not multiples of 128), and 16-byte
    loads from rows of an odd leading dimension: normwise residual, |L| <= 1,
    legal interchanges (a uniform matrix pivots in most columns)."""
    A = D.spd_bbt(n, seed=2, device=DEV) if recipe == "spd" else D.uniform01(n, seed=2, device=DEV)
    F = A.clone()
    ipiv, info = mlu.getrf(F, variant="la", nb=256, nb_inner=16)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    res, lmax = properties(A, F, ipiv)
    print(f"la n={n} {recipe}: residual {res:.2e}, max|L| {lmax:.3f}", flush=True)
    assert res <= (1e-13 if recipe == "spd" else 1e-12) and lmax <= 1.0
    del F, A
    torch.cuda.empty_cache()


# ------------------------------------------------------------ worker sharing on and off
@pytest.mark.parametrize("n,nb,recipe", [(3001, 64, "uniform"), (16384, 256, "spd")])
def test_la_without_worker_sharing_is_bitwise_la(n, nb, recipe):
    """MLU_LA_NOWS (the panel's workgroups do not join RU2 after PF3) does the
    same arithmetic as MLU_LA: every tile is computed the same way whichever
    workgroup takes it, so the factors and pivots are bit-identical."""
    A = D.spd_bbt(n, seed=4, device=DEV) if recipe == "spd" else D.uniform01(n, seed=4, device=DEV)
    F1, F2 = A.clone(), A.clone()
    ip1, in1 = mlu.getrf(F1, variant="la", nb=nb, nb_inner=16)
    ip2, in2 = mlu.getrf(F2, variant="la_nows", nb=nb, nb_inner=16)
    torch.cuda.synchronize()
    assert int(in1.item()) == 0 and int(in2.item()) == 0
    assert torch.equal(ip1, ip2) and torch.equal(F1, F2)
    del F1, F2, A
    torch.cuda.empty_cache()


# ------------------------------------------------------------ LA under graph capture
def test_la_graph_capture_replays_bit_equal():
    n, nb = 1500, 128
    A = dev(G.uniform01(n, seed=23))
    work = mlu.workspace(DEV)   # also prepares the library stream, before the capture
    ipiv_e = torch.empty(n, dtype=torch.int32, device=DEV)
    info_e = torch.empty(1, dtype=torch.int32, device=DEV)
    Fe = A.clone()
    mlu.getrf(Fe, variant="la", nb=nb, ipiv=ipiv_e, info=info_e, work=work)
    torch.cuda.synchronize()
    assert int(info_e.item()) == 0

    Fg = torch.empty_like(A)
    ipiv_g = torch.empty(n, dtype=torch.int32, device=DEV)
    info_g = torch.empty(1, dtype=torch.int32, device=DEV)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):   # the current stream inside is the capturing stream
        Fg.copy_(A)
        mlu.getrf(Fg, variant="la", nb=nb, ipiv=ipiv_g, info=info_g, work=work)
    torch.cuda.synchronize()
    other = dev(G.uniform01(700, seed=24))
    for rep in range(4):
        Fg.fill_(float("nan"))
        ipiv_g.fill_(-5)
        info_g.fill_(-5)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(Fg, Fe), f"replay {rep}: factors differ from the eager call"
        assert torch.equal(ipiv_g, ipiv_e) and int(info_g.item()) == 0
        # the program's own eager work between the replays
        X = other.clone()
        mlu.getrf(X, variant="la", nb=64)
        torch.cuda.synchronize()


# ------------------------------------------------------------ LU-IR divergence
def test_lu_ir_stops_when_corrections_diverge():
    n = 2048
    A = G.haar_spectrum(n, 1e5, seed=7)
    B = G.gaussian_rhs(n, 1, seed=1)
    X, ipiv, info, iters, berr = mlu.gesv_ir(dev(A), dev(B), precision="bf16", tol=1e-13, max_iter=30,
                                             variant="la", nb=128)
    torch.cuda.synchronize()
    it, be = int(iters.item()), float(berr.item())
    x = host(X)
    print(f"bf16 kappa=1e5 n={n}: iters {it}, berr {be:.2e}, max|x| {np.abs(x).max():.2e}", flush=True)
    assert int(info.item()) == 0
    if it == -1:   # not converged: stopped on divergence, with a finite, bounded iterate
        assert np.isfinite(be) and be < 1e-1 and np.all(np.isfinite(x))
    else:
        assert be <= 1e-13


# ------------------------------------------------------------ the 32-column diagonal-block kernel
def getf2(A):
    dA = dev(A)
    ipiv, info = mlu.getf2_block(dA)
    bw = A.shape[1]
    return host(dA), (host(ipiv)[:bw] - 1).tolist(), int(host(info)[0])


@pytest.mark.parametrize("m", [17, 32, 63, 64, 65, 300, 512, 513, 1024, 1025, 3000, 8192])
@pytest.mark.parametrize("bw", [17, 24, 32])
def test_wide_block_uniform(m, bw):
    if bw > m:
        pytest.skip("bw > m")
    A = G.uniform01(m, bw, seed=m + 3 * bw)
    F, piv, info = getf2(A)
    R = A.copy()
    opiv = O.lu_unb(R)
    assert info == 0
    assert piv == opiv
    assert np.abs(F - R).max() <= 1e-13 * max(1.0, np.abs(R).max())


@pytest.mark.parametrize("m,bw", [(40, 32), (2000, 32), (5000, 24), (8192, 32)])
def test_wide_block_known_answer_exact(m, bw):
    A, perm, L, U = G.known_answer(m, bw, seed=m + bw)
    F, piv, info = getf2(A)
    R = A.copy()
    opiv = O.lu_unb(R)
    assert info == 0 and piv == opiv
    assert np.array_equal(F, R)


@pytest.mark.parametrize("m,bw,fail_at", [(3000, 32, None), (3000, 32, 0), (3000, 32, 13), (3000, 32, 31),
                                          (8192, 32, 20), (300, 24, 9), (1000, 32, None)])
def test_wide_block_speculation_paths(m, bw, fail_at):
    # as for the 16-column kernel: pivots guessed from the leader's rows; rows
    # placed below them make the guess fail at column fail_at, and the block
    # is redone exactly; every path gives the partial-pivoting factors, bit
    # for bit on this exact input
    perm = G.leader_perm(m, bw, 64, fail_at, seed=m + bw)
    A, perm, L, U = G.known_answer(m, bw, seed=m, perm=perm)
    F, piv, info = getf2(A)
    R = A.copy()
    opiv = O.lu_unb(R)
    assert info == 0 and piv == opiv
    assert np.array_equal(F, R)
    assert np.array_equal(O.permutation_of(piv, m)[:bw], perm[:bw])


def test_wide_block_ties_and_zero_pivot():
    W = G.wilkinson_growth(32)
    F, piv, info = getf2(W)
    assert piv == list(range(32))
    R = W.copy()
    O.lu_unb(R)
    assert np.array_equal(F, R)
    Z = G.uniform01(700, 32, seed=3)
    Z[:, 5] = 0.0
    Z[:, 0] = 0.0
    F, piv, info = getf2(Z)
    R = Z.copy()
    inf_ = [0]
    opiv = O.lu_unb(R, info=inf_)
    assert info == 1 == inf_[0]
    assert piv == opiv
    assert np.abs(F - R).max() <= 1e-13


@pytest.mark.parametrize("variant", ["rl", "la", "ll"])
@pytest.mark.parametrize("inner", ["rl", "ll"])
def test_wide_blocks_inside_the_factorization(variant, inner):
    # b_i = 32 on a matrix short enough for the 32-column kernel (every panel
    # at most 8192 rows), pivoting at nearly every column
    n = 2100
    A = G.uniform01(n, seed=41)
    F, piv, info = gpu_getrf(A, variant, 128, 32, inner)
    R = A.copy()
    opiv, oinfo = O.getrf(R, variant, nb=128, inner=(inner, 32))
    assert info == oinfo == 0 and piv == opiv
    assert np.abs(F - R).max() <= 1e-11 * np.abs(R).max()
