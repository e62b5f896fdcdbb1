"""The C-ABI library loads and exports every symbol include/mlu.h declares;
host-side argument checks reject bad arguments before any device work.
CPU only: no call here reaches the GPU."""
import ctypes
import os
import re

import pytest

from paper_1611_06365_amd import mlu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mlu.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mlu_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(mlu.LIB_PATH):
        from paper_1611_06365_amd import build

        build.build()
    return mlu.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("mlu_dgetrf", "mlu_dgetrf_workspace", "mlu_dtrsm", "mlu_dgetrs", "mlu_dgemm_update",
                     "mlu_dlaswp", "mlu_dgetf2_block", "mlu_version", "mlu_trace_begin", "mlu_trace_end"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) == set(mlu.EXPORTED)


def test_version_and_workspace(lib):
    assert mlu.mlu_version() == 200
    rc, nbytes = mlu.mlu_dgetrf_workspace(16384, 16384, mlu.MLU_LA, 256, 16)
    assert rc == 0 and 0 < nbytes <= 1 << 20
    assert mlu.mlu_dgetrf_workspace(-1, 4, 0, 1, 0)[0] == -1
    assert mlu.mlu_dgetrf_workspace(4, 4, 7, 1, 0)[0] == -3
    assert mlu.mlu_dgetrf_workspace(4, 4, 0, 0, 0)[0] == -4
    assert mlu.mlu_dgetrf_workspace(4, 4, 0, 8, 33)[0] == -5
    assert mlu.mlu_dgetrf_workspace(4, 4, 0, 8, 32)[0] == 0


def _getrf(**kw):
    args = dict(stream=None, m=8, n=8, dA=1024, lda=8, d_ipiv=2048, d_info=4096, variant=0, nb=4, nb_inner=0,
                inner=0, h_schedule=None, n_schedule=0, iters_limit=-1, d_work=8192, work_bytes=1 << 20)
    args.update(kw)
    return mlu.mlu_dgetrf(*args.values())


@pytest.mark.parametrize("kw,code", [
    (dict(m=-1), -2), (dict(n=-3), -3), (dict(dA=None), -4), (dict(lda=7), -5), (dict(d_ipiv=None), -6),
    (dict(d_info=None), -7), (dict(variant=3), -8), (dict(variant=5), -8), (dict(variant=-1), -8),
    (dict(variant=4, nb=0), -9), (dict(nb=0), -9), (dict(nb_inner=33), -10),
    (dict(nb_inner=-1), -10), (dict(inner=2), -11), (dict(inner=-1), -11), (dict(iters_limit=-2), -14),
    (dict(d_work=None), -15), (dict(work_bytes=16), -16),
])
def test_getrf_argument_checks(lib, kw, code):
    assert _getrf(**kw) == code


def test_getrf_bad_schedule(lib):
    arr = (ctypes.c_int32 * 3)(4, 0, 4)
    assert _getrf(h_schedule=ctypes.cast(arr, ctypes.c_void_p), n_schedule=3) == -12
    arr = (ctypes.c_int32 * 1)(4)
    assert _getrf(h_schedule=ctypes.cast(arr, ctypes.c_void_p), n_schedule=0) == -13


def test_other_argument_checks(lib):
    assert mlu.mlu_dtrsm(None, b"X", b"U", 4, 4, 1024, 4, 2048, 4) == -2
    assert mlu.mlu_dtrsm(None, b"L", b"Q", 4, 4, 1024, 4, 2048, 4) == -3
    assert mlu.mlu_dtrsm(None, b"L", b"U", 4, 4, 1024, 3, 2048, 4) == -7
    assert mlu.mlu_dgetrs(None, 4, 2, 1024, 3, 2048, 4096, 2) == -5
    assert mlu.mlu_dgemm_update(None, 4, 4, 4, 1024, 3, 2048, 4, 4096, 4) == -6
    assert mlu.mlu_dlaswp(None, 4, 4, 1024, 4, 2, 1, 2048, None) == -7
    assert mlu.mlu_dgetf2_block(None, 40, 33, 1024, 33, 2048, 4096, 8192, 1 << 20) == -3
    assert mlu.mlu_dgetf2_block(None, 8193, 17, 1024, 17, 2048, 4096, 8192, 1 << 20) == -2
    assert mlu.mlu_dgetf2_block(None, 4, 8, 1024, 8, 2048, 4096, 8192, 1 << 20) == -3


def test_mixed_argument_checks(lib):
    import ctypes

    from paper_1611_06365_amd import mlu

    out = ctypes.c_size_t(0)
    assert lib.mlu_dsgesv_ir_workspace(-1, 1, ctypes.byref(out)) == -1
    assert lib.mlu_dsgesv_ir_workspace(4, -1, ctypes.byref(out)) == -2
    assert lib.mlu_dsgesv_ir_workspace(4, 1, None) == -3
    assert lib.mlu_dsgesv_ir_workspace(1000, 2, ctypes.byref(out)) == 0
    assert out.value >= 1000 * 1000 * 8 + 1000 * 2 * 8
    # argument checks return before anything is enqueued (no GPU needed)
    args = dict(stream=None, n=4, nrhs=1, dA=8, lda=4, dB=8, ldb=1, dX=8, ldx=1, precision=1, tol=1e-13,
                max_iter=5, variant=0, nb=2, nb_inner=0, d_ipiv=8, d_info=8, d_iters=8, d_berr=8, d_work=8,
                work_bytes=1 << 40)
    for key, bad, code in [("precision", 7, -10), ("tol", -1.0, -11), ("max_iter", -1, -12), ("variant", 9, -13),
                           ("nb", 0, -14), ("nb_inner", 33, -15), ("work_bytes", 16, -21), ("lda", 3, -5)]:
        kw = dict(args)
        kw[key] = bad
        assert mlu.mlu_dsgesv_ir(*kw.values()) == code, key
    # mlu_dsgetrf: precision is argument 12, later arguments shift by one
    g = dict(stream=None, m=4, n=4, dA=8, lda=4, d_ipiv=8, d_info=8, variant=0, nb=2, nb_inner=0, inner=0,
             precision=1, h_schedule=None, n_schedule=0, iters_limit=-1, d_work=8, work_bytes=16)
    kw = dict(g)
    kw["precision"] = 5
    assert mlu.mlu_dsgetrf(*kw.values()) == -12
    kw = dict(g)
    kw["inner"] = 2
    assert mlu.mlu_dsgetrf(*kw.values()) == -11
    assert mlu.mlu_dsgetrf(*g.values()) == -17      # workspace too small: argument 17
    kw = dict(g)
    kw["iters_limit"] = -2
    assert mlu.mlu_dsgetrf(*kw.values()) == -15


def test_batched_argument_checks(lib):
    import ctypes

    from paper_1611_06365_amd import mlu

    out = ctypes.c_size_t(0)
    assert lib.mlu_getrf_batched_workspace(-1, ctypes.byref(out)) == -1
    assert lib.mlu_getrf_batched_workspace(10, None) == -2
    assert lib.mlu_getrf_batched_workspace(20000, ctypes.byref(out)) == 0 and out.value >= 20000 * 4
    base = dict(stream=None, batch=2, d_n=8, d_A=8, d_lda=8, d_ipiv=8, d_info=8, max_n=64, nb=0, d_work=8,
                work_bytes=1 << 20)
    for fn in (mlu.mlu_dgetrf_batched, mlu.mlu_sgetrf_batched):
        for key, bad, code in [("batch", -1, -2), ("d_n", None, -3), ("d_A", None, -4), ("d_lda", None, -5),
                               ("d_ipiv", None, -6), ("d_info", None, -7), ("max_n", 513, -8),
                               ("nb", 24, -9), ("d_work", None, -10), ("work_bytes", 4, -11)]:
            kw = dict(base)
            kw[key] = bad
            assert fn(*kw.values()) == code, (fn.__name__, key)
        kw = dict(base)
        kw["batch"] = 0
        assert fn(*kw.values()) == 0


def test_et_argument_checks(lib):
    import ctypes

    from paper_1611_06365_amd import mlu

    cnt = ctypes.c_int(-5)
    base = dict(stream=None, m=4, n=4, dA=8, lda=4, d_ipiv=8, d_info=8, nb=2, nb_inner=0, force=0, min_width=0,
                h_widths=None, max_widths=0, n_widths=ctypes.cast(ctypes.byref(cnt), ctypes.c_void_p), d_work=8, work_bytes=1 << 40)
    for key, bad, code in [("m", -1, -2), ("n", -1, -3), ("dA", None, -4), ("lda", 3, -5), ("d_ipiv", None, -6),
                           ("d_info", None, -7), ("nb", 0, -8), ("nb_inner", 33, -9), ("force", 3, -10),
                           ("min_width", -1, -11), ("max_widths", 4, -12), ("max_widths", -1, -13),
                           ("n_widths", None, -14), ("d_work", None, -15), ("work_bytes", 16, -16)]:
        kw = dict(base)
        kw[key] = bad
        assert mlu.mlu_dgetrf_et(*kw.values()) == code, key


def test_gmres_ir_argument_checks(lib):
    out = ctypes.c_size_t(0)
    assert mlu.mlu_dsgesv_gmres_ir_workspace(-1, 8)[0] == -1
    assert mlu.mlu_dsgesv_gmres_ir_workspace(4, 0)[0] == -2
    assert mlu.mlu_dsgesv_gmres_ir_workspace(4, mlu.MLU_GMRES_MAX_KRYLOV + 1)[0] == -2
    assert lib.mlu_dsgesv_gmres_ir_workspace(4, 8, None) == -3
    rc, small = mlu.mlu_dsgesv_gmres_ir_workspace(100, 8)
    rc2, big = mlu.mlu_dsgesv_gmres_ir_workspace(100, 64)
    assert rc == rc2 == 0 and big > small >= 100 * 100 * 8 + 9 * 100 * 8
    o, i, b = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_double(0.0)
    addr = lambda v: ctypes.addressof(v)  # noqa: E731
    base = dict(stream=None, n=4, dA=8, lda=4, db=8, dx=8, precision=1, solver=1, tol=1e-13, max_outer=3,
                max_krylov=8, gmres_tol=1e-6, variant=2, nb=2, nb_inner=0, d_ipiv=8, d_info=8, h_outer=addr(o),
                h_inner=addr(i), h_berr=addr(b), d_work=8, work_bytes=1 << 40)
    for key, bad, code in [("n", -1, -2), ("n", 40000, -2), ("dA", None, -3), ("lda", 3, -4), ("db", None, -5),
                           ("dx", None, -6), ("precision", 3, -7), ("solver", 3, -8), ("tol", -1.0, -9),
                           ("tol", float("nan"), -9), ("max_outer", -1, -10), ("max_krylov", 0, -11),
                           ("max_krylov", mlu.MLU_GMRES_MAX_KRYLOV + 1, -11), ("gmres_tol", -1.0, -12),
                           ("variant", 3, -13), ("nb", 0, -14), ("nb_inner", 33, -15), ("d_ipiv", None, -16),
                           ("d_info", None, -17), ("h_outer", None, -18), ("h_inner", None, -19),
                           ("h_berr", None, -20), ("d_work", None, -21), ("work_bytes", 16, -22)]:
        kw = dict(base)
        kw[key] = bad
        assert mlu.mlu_dsgesv_gmres_ir(*kw.values()) == code, key


def test_noalloc_argument_checks(lib):
    base = dict(stream=None, m=8, n=8, dA=1024, lda=8, d_ipiv=2048, d_info=4096, variant=2, nb=4, nb_inner=0,
                inner=0, h_schedule=None, n_schedule=0, iters_limit=-1)
    for key, bad, code in [("m", -1, -2), ("m", 40000, -2), ("n", -1, -3), ("dA", None, -4), ("lda", 7, -5),
                           ("d_ipiv", None, -6), ("d_info", None, -7), ("variant", 3, -8), ("nb", 0, -9),
                           ("nb_inner", 33, -10), ("inner", 2, -11), ("iters_limit", -2, -14)]:
        kw = dict(base)
        kw[key] = bad
        assert mlu.mlu_dgetrf_noalloc(*kw.values()) == code, key
    arr = (ctypes.c_int32 * 2)(4, 0)
    kw = dict(base, h_schedule=ctypes.cast(arr, ctypes.c_void_p), n_schedule=2)
    assert mlu.mlu_dgetrf_noalloc(*kw.values()) == -12
    kw = dict(base, h_schedule=ctypes.cast(arr, ctypes.c_void_p), n_schedule=0)
    assert mlu.mlu_dgetrf_noalloc(*kw.values()) == -13
    if os.environ.get("HIP_VISIBLE_DEVICES", None) == "" or not _has_gpu():
        # no device here: nothing was set up, and nothing is enqueued
        assert mlu.mlu_dgetrf_noalloc(*base.values()) == mlu.MLU_ERR_NOINIT


def _has_gpu():
    try:
        import torch

        return torch.cuda.device_count() > 0
    except Exception:
        return False
