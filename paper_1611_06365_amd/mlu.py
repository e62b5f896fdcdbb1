"""ctypes binding of libmlu (include/mlu.h): argument marshalling only.

Every function here has the name and argument order of the C entry point; the
helpers at the bottom only turn torch tensors into pointers, sizes and the
current HIP stream.  All computation happens in the HIP kernels of libmlu.so;
if the library is not built this module raises on import of any entry point.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmlu.so")

MLU_RL, MLU_LL, MLU_LA, MLU_LA_NOWS = 0, 1, 2, 4
VARIANT_IDS = {"rl": MLU_RL, "ll": MLU_LL, "la": MLU_LA, "la_nows": MLU_LA_NOWS}
MLU_ERR_HIP = -1000
MLU_ERR_NOINIT = -1001
MLU_INFO_SYNC_TIMEOUT = -999
MLU_INFO_BAD_PIVOT = -998
MLU_MAX_NB_INNER = 32
MLU_PREC_FP64, MLU_PREC_FP32, MLU_PREC_BF16 = 0, 1, 2
PRECISION_IDS = {"fp64": MLU_PREC_FP64, "fp32": MLU_PREC_FP32, "bf16": MLU_PREC_BF16}
MLU_IR_LU, MLU_IR_GMRES, MLU_IR_AUTO = 0, 1, 2
IR_SOLVER_IDS = {"lu": MLU_IR_LU, "gmres": MLU_IR_GMRES, "auto": MLU_IR_AUTO}
MLU_GMRES_MAX_KRYLOV = 512

_vp, _i, _sz, _c = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t, ctypes.c_char

_SIGNATURES = {
    "mlu_version": ([], _i),
    "mlu_init": ([], _i),
    "mlu_dgetrf_workspace": ([_i, _i, _i, _i, _i, ctypes.POINTER(_sz)], _i),
    "mlu_dgetrf": ([_vp, _i, _i, _vp, _i, _vp, _vp, _i, _i, _i, _i, _vp, _i, _i, _vp, _sz], _i),
    "mlu_dgetrf_noalloc": ([_vp, _i, _i, _vp, _i, _vp, _vp, _i, _i, _i, _i, _vp, _i, _i], _i),
    "mlu_dsgetrf": ([_vp, _i, _i, _vp, _i, _vp, _vp, _i, _i, _i, _i, _i, _vp, _i, _i, _vp, _sz], _i),
    "mlu_select": ([_vp, _i, _i, _i, _i, _vp, _vp, _vp], _i),
    "mlu_dgetrf_et": ([_vp, _i, _i, _vp, _i, _vp, _vp, _i, _i, _i, _i, _vp, _i, _vp, _vp, _sz], _i),
    "mlu_dsgesv_ir_workspace": ([_i, _i, ctypes.POINTER(_sz)], _i),
    "mlu_dsgesv_ir": ([_vp, _i, _i, _vp, _i, _vp, _i, _vp, _i, _i, ctypes.c_double, _i, _i, _i, _i, _vp, _vp, _vp,
                       _vp, _vp, _sz], _i),
    "mlu_dsgesv_gmres_ir_workspace": ([_i, _i, ctypes.POINTER(_sz)], _i),
    "mlu_dsgesv_gmres_ir": ([_vp, _i, _vp, _i, _vp, _vp, _i, _i, ctypes.c_double, _i, _i, ctypes.c_double, _i, _i,
                             _i, _vp, _vp, _vp, _vp, _vp, _vp, _sz], _i),
    "mlu_getrf_batched_workspace": ([_i, ctypes.POINTER(_sz)], _i),
    "mlu_dgetrf_batched": ([_vp, _i, _vp, _vp, _vp, _vp, _vp, _i, _i, _vp, _sz], _i),
    "mlu_sgetrf_batched": ([_vp, _i, _vp, _vp, _vp, _vp, _vp, _i, _i, _vp, _sz], _i),
    "mlu_dtrsm": ([_vp, _c, _c, _i, _i, _vp, _i, _vp, _i], _i),
    "mlu_dgetrs": ([_vp, _i, _i, _vp, _i, _vp, _vp, _i], _i),
    "mlu_dgemm_update": ([_vp, _i, _i, _i, _vp, _i, _vp, _i, _vp, _i], _i),
    "mlu_dlaswp": ([_vp, _i, _i, _vp, _i, _i, _i, _vp, _vp], _i),
    "mlu_dgetf2_block": ([_vp, _i, _i, _vp, _i, _vp, _vp, _vp, _sz], _i),
    "mlu_trace_begin": ([_i], _i),
    "mlu_trace_end": ([ctypes.POINTER(_i), ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                       ctypes.POINTER(ctypes.c_double)], _i),
}
EXPORTED = tuple(_SIGNATURES)

_lib = None


def load(path: str = LIB_PATH):
    """Load libmlu.so (raises OSError if it has not been built)."""
    global _lib
    if _lib is None:
        try:  # bind to the HIP runtime torch already carries (same soname)
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(path):
            raise OSError(f"libmlu.so not found at {path}; run paper_1611_06365_amd/build.py")
        lib = ctypes.CDLL(path)
        for name, (args, res) in _SIGNATURES.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def _call(name, *args):
    return getattr(load(), name)(*args)


# ---------------------------------------------------------------- C entry points
def mlu_version() -> int:
    return _call("mlu_version")


def mlu_init() -> int:
    return _call("mlu_init")


def mlu_dgetrf_workspace(m, n, variant, nb, nb_inner) -> tuple[int, int]:
    out = _sz(0)
    rc = _call("mlu_dgetrf_workspace", m, n, variant, nb, nb_inner, ctypes.byref(out))
    return rc, out.value


def mlu_dgetrf(stream, m, n, dA, lda, d_ipiv, d_info, variant, nb, nb_inner, inner, h_schedule, n_schedule,
               iters_limit, d_work, work_bytes) -> int:
    return _call("mlu_dgetrf", stream, m, n, dA, lda, d_ipiv, d_info, variant, nb, nb_inner, inner, h_schedule,
                 n_schedule, iters_limit, d_work, work_bytes)


def mlu_dgetrf_noalloc(stream, m, n, dA, lda, d_ipiv, d_info, variant, nb, nb_inner, inner, h_schedule, n_schedule,
                       iters_limit) -> int:
    return _call("mlu_dgetrf_noalloc", stream, m, n, dA, lda, d_ipiv, d_info, variant, nb, nb_inner, inner,
                 h_schedule, n_schedule, iters_limit)


def mlu_dsgetrf(stream, m, n, dA, lda, d_ipiv, d_info, variant, nb, nb_inner, inner, precision, h_schedule,
                n_schedule, iters_limit, d_work, work_bytes) -> int:
    return _call("mlu_dsgetrf", stream, m, n, dA, lda, d_ipiv, d_info, variant, nb, nb_inner, inner, precision,
                 h_schedule, n_schedule, iters_limit, d_work, work_bytes)


def mlu_dsgesv_ir_workspace(n, nrhs) -> tuple[int, int]:
    out = _sz(0)
    rc = _call("mlu_dsgesv_ir_workspace", n, nrhs, ctypes.byref(out))
    return rc, out.value


def mlu_dsgesv_ir(stream, n, nrhs, dA, lda, dB, ldb, dX, ldx, precision, tol, max_iter, variant, nb, nb_inner,
                  d_ipiv, d_info, d_iters, d_berr, d_work, work_bytes) -> int:
    return _call("mlu_dsgesv_ir", stream, n, nrhs, dA, lda, dB, ldb, dX, ldx, precision, tol, max_iter, variant, nb,
                 nb_inner, d_ipiv, d_info, d_iters, d_berr, d_work, work_bytes)


def mlu_dsgesv_gmres_ir_workspace(n, max_krylov) -> tuple[int, int]:
    out = _sz(0)
    rc = _call("mlu_dsgesv_gmres_ir_workspace", n, max_krylov, ctypes.byref(out))
    return rc, out.value


def mlu_dsgesv_gmres_ir(stream, n, dA, lda, db, dx, precision, solver, tol, max_outer, max_krylov, gmres_tol,
                        variant, nb, nb_inner, d_ipiv, d_info, h_outer, h_inner, h_berr, d_work, work_bytes) -> int:
    return _call("mlu_dsgesv_gmres_ir", stream, n, dA, lda, db, dx, precision, solver, tol, max_outer, max_krylov,
                 gmres_tol, variant, nb, nb_inner, d_ipiv, d_info, h_outer, h_inner, h_berr, d_work, work_bytes)


def mlu_getrf_batched_workspace(batch) -> tuple[int, int]:
    out = _sz(0)
    rc = _call("mlu_getrf_batched_workspace", batch, ctypes.byref(out))
    return rc, out.value


def mlu_dgetrf_batched(stream, batch, d_n, d_A, d_lda, d_ipiv, d_info, max_n, nb, d_work, work_bytes) -> int:
    return _call("mlu_dgetrf_batched", stream, batch, d_n, d_A, d_lda, d_ipiv, d_info, max_n, nb, d_work, work_bytes)


def mlu_sgetrf_batched(stream, batch, d_n, d_A, d_lda, d_ipiv, d_info, max_n, nb, d_work, work_bytes) -> int:
    return _call("mlu_sgetrf_batched", stream, batch, d_n, d_A, d_lda, d_ipiv, d_info, max_n, nb, d_work, work_bytes)


def mlu_dtrsm(stream, uplo, diag, m, nrhs, dT, ldt, dB, ldb) -> int:
    return _call("mlu_dtrsm", stream, uplo, diag, m, nrhs, dT, ldt, dB, ldb)


def mlu_dgetrs(stream, n, nrhs, dLU, lda, d_ipiv, dB, ldb) -> int:
    return _call("mlu_dgetrs", stream, n, nrhs, dLU, lda, d_ipiv, dB, ldb)


def mlu_dgemm_update(stream, m, n, k, dA, lda, dB, ldb, dC, ldc) -> int:
    return _call("mlu_dgemm_update", stream, m, n, k, dA, lda, dB, ldb, dC, ldc)


def mlu_dlaswp(stream, m, ncols, dA, lda, k1, k2, d_ipiv, d_info) -> int:
    return _call("mlu_dlaswp", stream, m, ncols, dA, lda, k1, k2, d_ipiv, d_info)


def mlu_dgetf2_block(stream, m, bw, dA, lda, d_ipiv, d_info, d_work, work_bytes) -> int:
    return _call("mlu_dgetf2_block", stream, m, bw, dA, lda, d_ipiv, d_info, d_work, work_bytes)


def mlu_trace_begin(capacity) -> int:
    return _call("mlu_trace_begin", capacity)


def mlu_trace_end() -> tuple[int, int, float, float, float]:
    n, ms, fl, by = _i(0), ctypes.c_double(0), ctypes.c_double(0), ctypes.c_double(0)
    rc = _call("mlu_trace_end", ctypes.byref(n), ctypes.byref(ms), ctypes.byref(fl), ctypes.byref(by))
    return rc, n.value, ms.value, fl.value, by.value


# ---------------------------------------------------------------- torch marshalling
class MluError(RuntimeError):
    pass


def check(rc: int, what: str) -> None:
    if rc != 0:
        raise MluError(f"{what} returned {rc}")


def _stream(stream=None) -> int:
    import torch

    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


def _rowmajor(t, name):
    import torch

    if t.dtype != torch.float64 or not t.is_cuda or t.dim() != 2 or t.stride(1) != 1:
        raise ValueError(f"{name} must be a 2-D float64 CUDA tensor with unit column stride")
    return t.data_ptr(), max(1, t.stride(0))


def _i32(t, name, n):
    import torch

    if t.dtype != torch.int32 or not t.is_cuda or not t.is_contiguous() or t.numel() < n:
        raise ValueError(f"{name} must be a contiguous int32 CUDA tensor with >= {n} entries")
    return t.data_ptr()


def workspace(device=None):
    """A device workspace tensor large enough for mlu_dgetrf."""
    import torch

    rc, nbytes = mlu_dgetrf_workspace(1, 1, MLU_RL, 1, 0)
    check(rc, "mlu_dgetrf_workspace")
    return torch.empty(nbytes, dtype=torch.uint8, device=device or "cuda")


def getrf(A, variant="rl", nb=256, nb_inner=0, schedule=None, iters_limit=-1, ipiv=None, info=None,
          work=None, stream=None, precision="fp64", inner="rl"):
    """Factor A (m x n float64 CUDA tensor, row-major) in place; returns (ipiv, info) tensors.

    inner: "rl" or "ll", the algorithm of the panel factorization.
    precision="fp32" / "bf16" calls mlu_dsgetrf (lower-precision products in
    the outer trailing updates).  No synchronization: read info after the
    stream has finished.
    """
    import torch

    pa, lda = _rowmajor(A, "A")
    m, n = A.shape
    k = min(m, n)
    ipiv = torch.empty(max(k, 1), dtype=torch.int32, device=A.device) if ipiv is None else ipiv
    info = torch.empty(1, dtype=torch.int32, device=A.device) if info is None else info
    work = workspace(A.device) if work is None else work
    sched = None
    nsched = 0
    if schedule is not None:
        arr = (ctypes.c_int32 * len(schedule))(*[int(b) for b in schedule])
        sched, nsched = ctypes.cast(arr, ctypes.c_void_p), len(schedule)
    v = VARIANT_IDS[variant] if isinstance(variant, str) else int(variant)
    iv = VARIANT_IDS[inner] if isinstance(inner, str) else int(inner)
    if precision == "fp64":
        rc = mlu_dgetrf(_stream(stream), m, n, pa, lda, _i32(ipiv, "ipiv", k), _i32(info, "info", 1), v, nb,
                        nb_inner, iv, sched, nsched, iters_limit, work.data_ptr(), work.numel())
        check(rc, "mlu_dgetrf")
    else:
        rc = mlu_dsgetrf(_stream(stream), m, n, pa, lda, _i32(ipiv, "ipiv", k), _i32(info, "info", 1), v, nb,
                         nb_inner, iv, PRECISION_IDS[precision], sched, nsched, iters_limit, work.data_ptr(),
                         work.numel())
        check(rc, "mlu_dsgetrf")
    return ipiv, info


VARIANT_NAMES = {0: "rl", 1: "ll", 2: "la", 3: "batched"}


def packed_model(model):
    """A packed float list (selector.pack) as the ctypes array mlu_select reads."""
    return (ctypes.c_float * len(model))(*model)


def select(n, precision="fp64", model=None, batch=1, with_fallback=False):
    """The learned selector through the C ABI (mlu_select): (variant, nb) for
    `batch` matrices of order n ("batched" with the panel width for a batch of
    small matrices); with_fallback=True adds whether the model defers to the
    autotuner.  `model`: a packed float list (selector.pack) or a
    packed_model() array; default, the package's trained model."""
    arr = _packed_default() if model is None else (model if isinstance(model, ctypes.Array) else
                                                    packed_model(model))
    v, nb, fb = ctypes.c_int(-1), ctypes.c_int(-1), ctypes.c_int(-1)
    rc = _call("mlu_select", ctypes.cast(arr, ctypes.c_void_p), len(arr), int(n), int(batch),
               PRECISION_IDS[precision], ctypes.cast(ctypes.byref(v), ctypes.c_void_p),
               ctypes.cast(ctypes.byref(nb), ctypes.c_void_p), ctypes.cast(ctypes.byref(fb), ctypes.c_void_p))
    check(rc, "mlu_select")
    out = (VARIANT_NAMES[v.value], nb.value)
    return (*out, bool(fb.value)) if with_fallback else out


_PACKED = None


def _packed_default():
    global _PACKED
    if _PACKED is None:
        import json

        from . import selector

        with open(selector.MODEL_PATH) as f:
            _PACKED = packed_model(selector.pack(json.load(f)))
    return _PACKED


ET_FORCE_IDS = {"signal": 0, "always": 1, "never": 2}


def mlu_dgetrf_et(stream, m, n, dA, lda, d_ipiv, d_info, nb, nb_inner, force, min_width, h_widths, max_widths,
                  n_widths, d_work, work_bytes) -> int:
    return _call("mlu_dgetrf_et", stream, m, n, dA, lda, d_ipiv, d_info, nb, nb_inner, force, min_width, h_widths,
                 max_widths, n_widths, d_work, work_bytes)


def getrf_et(A, nb=256, nb_inner=0, force="signal", min_width=0, ipiv=None, info=None, work=None, stream=None):
    """Factor A in place by look-ahead LU with early termination of the panel
    (mlu_dgetrf_et); returns (ipiv, info, widths) with widths the realized
    panel widths (a host list).  The call waits on the device once per outer
    iteration."""
    import torch

    pa, lda = _rowmajor(A, "A")
    m, n = A.shape
    k = min(m, n)
    ipiv = torch.empty(max(k, 1), dtype=torch.int32, device=A.device) if ipiv is None else ipiv
    info = torch.empty(1, dtype=torch.int32, device=A.device) if info is None else info
    work = workspace(A.device) if work is None else work
    cap = max(k, 1)
    arr = (ctypes.c_int32 * cap)()
    cnt = ctypes.c_int(0)
    rc = mlu_dgetrf_et(_stream(stream), m, n, pa, lda, _i32(ipiv, "ipiv", k), _i32(info, "info", 1), nb, nb_inner,
                       ET_FORCE_IDS[force], min_width, ctypes.cast(arr, ctypes.c_void_p), cap,
                       ctypes.cast(ctypes.byref(cnt), ctypes.c_void_p), work.data_ptr(), work.numel())
    check(rc, "mlu_dgetrf_et")
    return ipiv, info, [int(arr[i]) for i in range(min(cnt.value, cap))]


def gesv_ir(A, B, precision="fp32", tol=1e-13, max_iter=10, variant="la", nb=256, nb_inner=0, X=None, work=None,
            stream=None):
    """Solve A X = B by mixed-precision LU and FP64 refinement (mlu_dsgesv_ir).

    Returns (X, ipiv, info, iters, berr); iters, berr and info are device
    tensors, valid once the stream has finished.  A and B are not modified.
    """
    import torch

    pa, lda = _rowmajor(A, "A")
    pb, ldb = _rowmajor(B, "B")
    n, nrhs = A.shape[0], B.shape[1]
    if A.shape[1] != n or B.shape[0] != n:
        raise ValueError("A must be n x n and B n x nrhs")
    X = torch.empty_like(B) if X is None else X
    px, ldx = _rowmajor(X, "X")
    if work is None:
        rc, nbytes = mlu_dsgesv_ir_workspace(n, nrhs)
        check(rc, "mlu_dsgesv_ir_workspace")
        work = torch.empty(nbytes, dtype=torch.uint8, device=A.device)
    ipiv = torch.empty(max(n, 1), dtype=torch.int32, device=A.device)
    info = torch.empty(1, dtype=torch.int32, device=A.device)
    iters = torch.empty(1, dtype=torch.int32, device=A.device)
    berr = torch.empty(1, dtype=torch.float64, device=A.device)
    v = VARIANT_IDS[variant] if isinstance(variant, str) else int(variant)
    rc = mlu_dsgesv_ir(_stream(stream), n, nrhs, pa, lda, pb, ldb, px, ldx, PRECISION_IDS[precision], tol,
                       max_iter, v, nb, nb_inner, ipiv.data_ptr(), info.data_ptr(), iters.data_ptr(),
                       berr.data_ptr(), work.data_ptr(), work.numel())
    check(rc, "mlu_dsgesv_ir")
    return X, ipiv, info, iters, berr


def gesv_gmres_ir(A, b, precision="fp32", solver="gmres", tol=1e-13, max_outer=10, max_krylov=64,
                  gmres_tol=1e-6, variant="la", nb=256, nb_inner=0, x=None, work=None, stream=None):
    """Solve A x = b by mixed-precision LU and FP64 refinement with GMRES
    corrections (mlu_dsgesv_gmres_ir).  b is a length-n FP64 vector.

    Returns (x, ipiv, info, outer, inner, berr): outer, inner and berr are host
    values (the call waits for the stream); ipiv and info are device tensors.
    A and b are not modified.
    """
    import torch

    pa, lda = _rowmajor(A, "A")
    n = A.shape[0]
    if A.shape[1] != n or b.dim() != 1 or b.shape[0] != n:
        raise ValueError("A must be n x n and b of length n")
    if b.dtype != torch.float64 or not b.is_contiguous() or b.device != A.device:
        raise ValueError("b must be a contiguous float64 vector on A's device")
    x = torch.empty_like(b) if x is None else x
    if x.dtype != torch.float64 or not x.is_contiguous() or x.shape != b.shape or x.device != A.device:
        raise ValueError("x must be a contiguous float64 vector like b")
    if work is None:
        rc, nbytes = mlu_dsgesv_gmres_ir_workspace(n, max_krylov)
        check(rc, "mlu_dsgesv_gmres_ir_workspace")
        work = torch.empty(nbytes, dtype=torch.uint8, device=A.device)
    ipiv = torch.empty(max(n, 1), dtype=torch.int32, device=A.device)
    info = torch.empty(1, dtype=torch.int32, device=A.device)
    outer, inner, berr = _i(0), _i(0), ctypes.c_double(0.0)
    v = VARIANT_IDS[variant] if isinstance(variant, str) else int(variant)
    rc = mlu_dsgesv_gmres_ir(_stream(stream), n, pa, lda, b.data_ptr(), x.data_ptr(), PRECISION_IDS[precision],
                             IR_SOLVER_IDS[solver], tol, max_outer, max_krylov, gmres_tol, v, nb, nb_inner,
                             ipiv.data_ptr(), info.data_ptr(), ctypes.addressof(outer), ctypes.addressof(inner),
                             ctypes.addressof(berr), work.data_ptr(), work.numel())
    check(rc, "mlu_dsgesv_gmres_ir")
    return x, ipiv, info, outer.value, inner.value, berr.value


def trsm(T, B, uplo="L", diag="U", stream=None):
    pt, ldt = _rowmajor(T, "T")
    pb, ldb = _rowmajor(B, "B")
    rc = mlu_dtrsm(_stream(stream), uplo.encode(), diag.encode(), T.shape[0], B.shape[1], pt, ldt, pb, ldb)
    check(rc, "mlu_dtrsm")


def getrs(LU, ipiv, B, stream=None):
    pa, lda = _rowmajor(LU, "LU")
    pb, ldb = _rowmajor(B, "B")
    n = LU.shape[0]
    rc = mlu_dgetrs(_stream(stream), n, B.shape[1], pa, lda, _i32(ipiv, "ipiv", n), pb, ldb)
    check(rc, "mlu_dgetrs")


def gemm_update(C, A, B, stream=None):
    pc, ldc = _rowmajor(C, "C")
    pa, lda = _rowmajor(A, "A")
    pb, ldb = _rowmajor(B, "B")
    m, k = A.shape
    n = B.shape[1]
    rc = mlu_dgemm_update(_stream(stream), m, n, k, pa, lda, pb, ldb, pc, ldc)
    check(rc, "mlu_dgemm_update")


def laswp(A, k1, k2, ipiv, info=None, stream=None):
    pa, lda = _rowmajor(A, "A")
    pinfo = info.data_ptr() if info is not None else None
    rc = mlu_dlaswp(_stream(stream), A.shape[0], A.shape[1], pa, lda, k1, k2, _i32(ipiv, "ipiv", k2), pinfo)
    check(rc, "mlu_dlaswp")


def getf2_block(A, ipiv=None, info=None, work=None, stream=None):
    import torch

    pa, lda = _rowmajor(A, "A")
    m, bw = A.shape
    ipiv = torch.empty(max(bw, 1), dtype=torch.int32, device=A.device) if ipiv is None else ipiv
    info = torch.empty(1, dtype=torch.int32, device=A.device) if info is None else info
    work = workspace(A.device) if work is None else work
    rc = mlu_dgetf2_block(_stream(stream), m, bw, pa, lda, _i32(ipiv, "ipiv", bw), _i32(info, "info", 1),
                          work.data_ptr(), work.numel())
    check(rc, "mlu_dgetf2_block")
    return ipiv, info


MLU_BATCH_MAX_N = 512


class BatchPlan:
    """Device arrays describing a batch of square matrices for mlu_?getrf_batched:
    orders, matrix pointers, leading dimensions, one int32 interchange buffer
    (with per-matrix pointers into it), info and the workspace.  Built once;
    the matrices it points to are factored in place by `run`."""

    def __init__(self, mats, max_n=None, nb=0):
        import torch

        if not mats:
            raise ValueError("empty batch")
        dt = mats[0].dtype
        if dt not in (torch.float64, torch.float32):
            raise ValueError("matrices must be float64 or float32")
        dev = mats[0].device
        ns, ptrs, ldas = [], [], []
        for m in mats:
            if m.dtype != dt or m.device != dev or m.dim() != 2 or m.shape[0] != m.shape[1] or (
                    m.numel() and m.stride(1) != 1):
                raise ValueError("every matrix must be a square row-major tensor of the batch's dtype and device")
            ns.append(int(m.shape[0]))
            ptrs.append(int(m.data_ptr()))
            ldas.append(max(1, int(m.stride(0)) if m.numel() else 1))
        self.dtype, self.batch, self.nb = dt, len(mats), int(nb)
        self.max_n = max(ns) if max_n is None else int(max_n)
        offs = [0]
        for n in ns:
            offs.append(offs[-1] + max(n, 1))
        self.ipiv = torch.empty(offs[-1], dtype=torch.int32, device=dev)
        base = self.ipiv.data_ptr()
        self.offsets = offs
        self.d_n = torch.tensor(ns, dtype=torch.int32, device=dev)
        self.d_A = torch.tensor(ptrs, dtype=torch.int64, device=dev)
        self.d_lda = torch.tensor(ldas, dtype=torch.int32, device=dev)
        self.d_ipiv = torch.tensor([base + 4 * o for o in offs[:-1]], dtype=torch.int64, device=dev)
        self.info = torch.empty(len(mats), dtype=torch.int32, device=dev)
        rc, nbytes = mlu_getrf_batched_workspace(len(mats))
        check(rc, "mlu_getrf_batched_workspace")
        self.work = torch.empty(nbytes, dtype=torch.uint8, device=dev)

    def run(self, stream=None):
        import torch

        fn = mlu_dgetrf_batched if self.dtype == torch.float64 else mlu_sgetrf_batched
        rc = fn(_stream(stream), self.batch, self.d_n.data_ptr(), self.d_A.data_ptr(), self.d_lda.data_ptr(),
                self.d_ipiv.data_ptr(), self.info.data_ptr(), self.max_n, self.nb, self.work.data_ptr(), self.work.numel())
        check(rc, "mlu_getrf_batched")

    def pivots(self, i):
        return self.ipiv[self.offsets[i]:self.offsets[i + 1]]


BATCH_NB_CANDIDATES = (16, 32)


def tune_batched(mats, max_n=None, candidates=BATCH_NB_CANDIDATES, reps=2):
    """Choose the panel width of mlu_?getrf_batched for a batch by timing each
    candidate on scratch copies of the matrices (the inputs are untouched),
    on the current stream, the best of `reps` runs each.  Returns
    (best_nb, {nb: ms})."""
    import torch

    work = [m.clone() for m in mats]
    times = {}
    for nb in candidates:
        plan = BatchPlan(work, max_n, nb)
        best = float("inf")
        for _ in range(reps):
            for w, m in zip(work, mats):
                w.copy_(m)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            plan.run()
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        times[nb] = best
    return min(times, key=times.get), times


def getrf_batched(mats, max_n=None, stream=None, nb=0):
    """Factor every matrix of the list in place; returns the BatchPlan (its
    `info` and `pivots(i)` are valid once the stream has finished)."""
    plan = BatchPlan(mats, max_n, nb)
    plan.run(stream)
    return plan
