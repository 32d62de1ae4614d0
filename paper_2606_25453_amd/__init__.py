"""Python binding of libozk (FP64/complex128 GEMM emulated on MI355X INT8
MFMA with the Ozaki schemes).

Argument marshalling only: every function forwards to the C ABI of the same
name declared in include/ozk.h; all arithmetic runs in the library's HIP
kernels.  PyTorch supplies device memory (tensors) and streams.  There is no
fallback: importing works without a GPU, but every call needs the built
library (``paper_2606_25453_amd/libozk.so``) and raises if it is missing.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libozk.so")

OZK_OK = 0
OZK_ERR_INVALID_ARG = -1
OZK_ERR_UNSUPPORTED = -2
OZK_ERR_WORKSPACE = -3
OZK_ERR_HIP = -4
OZK_SCHEME1 = 1
OZK_SCHEME2 = 2
OZK_OP_DGEMM = 0
OZK_OP_ZGEMM = 1
OZK_OP_DGEMM_BATCHED = 2
OZK_F64, OZK_F32, OZK_C128, OZK_C64 = 0, 1, 2, 3
OZK_ROW_MAJOR, OZK_COL_MAJOR = 0, 1
OZK_OP_ZGEMM_BATCHED = 3
OZK_ROW_ALIGN = 256
OZK_K_CHUNK = 32
OZK_EXP_ZERO = -100000
OZK_EXP_NONFINITE = 100000
OZK_SELECTOR_PARAMS = 8220
OZK_SELECTOR_HEADS = 28
OZK_SELECTOR_COUNTERS = 34
OZK_SELECTOR_INFO = 8
OZK_MAX_ROWS = 1 << 24
OZK_S2_MAX_K = 1 << 22
OZK_S1_VARIANTS = 4
OZK_S2_VARIANTS = 7
OZK_S2_FUSED_CRT = 4
OZK_NOALLOC_SCRATCH_BYTES = 64 << 20
OZK_FLAG_NONFINITE = 1
OZK_FLAG_SELECTOR_FALLBACK = 2
OZK_FLAG_SCHEME2_CHOSEN = 4
OZK_FLAG_S_UNPROVEN = 8


class OzkGemmConfig(ctypes.Structure):
    """ozk_gemm_config: tile variant, raster order, raster group, K split."""
    _fields_ = [("variant", ctypes.c_int), ("raster", ctypes.c_int), ("group", ctypes.c_int),
                ("split", ctypes.c_int)]

    def as_tuple(self):
        return (self.variant, self.raster, self.group, self.split)

# every symbol include/ozk.h declares
EXPORTS = (
    "ozk_create", "ozk_destroy", "ozk_last_arg", "ozk_status_string", "ozk_version", "ozk_set_k_split",
    "ozk_s1_packed_bytes", "ozk_s2_packed_bytes", "ozk_s1_k_split", "ozk_workspace_size",
    "ozk_gemm_ex", "ozk_get_flags", "ozk_zgemm", "ozk_cgemm", "ozk_zgemm_auto", "ozk_batch_plan_tiles", "ozk_tune_batch", "ozk_s2_unfused_workspace_size", "ozk_s2_gemm_unfused",
    "ozk_dgemm", "ozk_dgemm_noalloc", "ozk_dgemm_t", "ozk_sgemm", "ozk_zgemm_3m", "ozk_cgemm_3m", "ozk_s1_dgemm_unfused", "ozk_s1_unfused_workspace_size", "ozk_s1_split_rows", "ozk_s1_split_cols", "ozk_s1_gemm",
    "ozk_s1_diagonals", "ozk_s2_split_rows", "ozk_s2_split_cols", "ozk_s2_gemm_mod", "ozk_s2_crt",
    "ozk_selector_load", "ozk_select", "ozk_dgemm_auto", "ozk_mlp_forward", "ozk_mlp_grad", "ozk_mlp_adam",
    "ozk_ref_dd", "ozk_batch_plan_create", "ozk_gemm_batched", "ozk_batch_plan_destroy",
    "ozk_config_set", "ozk_config_get", "ozk_config_clear", "ozk_config_save", "ozk_config_load",
    "ozk_tune_workspace_size", "ozk_tune",
)


class OzkError(RuntimeError):
    def __init__(self, fn: str, status: int, arg: int):
        self.status = status
        self.arg = arg
        msg = _lib().ozk_status_string(status).decode() if _LIB is not None else str(status)
        super().__init__("%s failed: %s (status %d, argument %d)" % (fn, msg, status, arg))


_LIB = None


def _lib() -> ctypes.CDLL:
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libozk.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    P, I, I64, D, SZ = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    sig = {
        "ozk_create": (I, [ctypes.POINTER(P), I]),
        "ozk_destroy": (I, [P]),
        "ozk_last_arg": (I, [P]),
        "ozk_status_string": (ctypes.c_char_p, [I]),
        "ozk_version": (ctypes.c_char_p, []),
        "ozk_set_k_split": (I, [P, I64]),
        "ozk_s1_packed_bytes": (SZ, [I64, I64, I]),
        "ozk_s2_packed_bytes": (SZ, [I64, I64, I, I]),
        "ozk_s1_k_split": (I64, [I]),
        "ozk_workspace_size": (I, [P, I, I, I64, I64, I64, I, ctypes.POINTER(SZ)]),
        "ozk_dgemm": (I, [P, I, I, I64, I64, I64, D, P, I64, P, I64, D, P, I64, P, SZ, P]),
        "ozk_get_flags": (I, [P, P, ctypes.POINTER(ctypes.c_uint32)]),
        "ozk_gemm_ex": (I, [P, I, I, I, I, I, I, I64, I64, I64, P, P, I64, P, I64, P, P, I64, P, SZ, P]),
        "ozk_batch_plan_tiles": (I, [P, I, P]),
        "ozk_tune_batch": (I, [P, P, P, SZ, I, P]),
        "ozk_zgemm_auto": (I, [P, D, I64, I64, I64, P, P, I64, P, I64, P, P, I64, P, SZ, P, P]),
        "ozk_zgemm": (I, [P, I, I, I64, I64, I64, P, P, I64, P, I64, P, P, I64, P, SZ, P]),
        "ozk_cgemm": (I, [P, I, I, I64, I64, I64, P, P, I64, P, I64, P, P, I64, P, SZ, P]),
        "ozk_s2_unfused_workspace_size": (I, [P, I, I, I64, I64, I64, ctypes.POINTER(SZ)]),
        "ozk_s2_gemm_unfused": (I, [P, I, I, I64, I64, I64, P, P, I64, P, I64, P, P, I64, P, SZ, P]),
        "ozk_dgemm_noalloc": (I, [P, I, I, I64, I64, I64, D, P, I64, P, I64, D, P, I64, P]),
        "ozk_dgemm_t": (I, [P, I, I, I, I, I64, I64, I64, D, P, I64, P, I64, D, P, I64, P, SZ, P]),
        "ozk_sgemm": (I, [P, I, I, I64, I64, I64, ctypes.c_float, P, I64, P, I64, ctypes.c_float, P, I64, P, SZ, P]),
        "ozk_cgemm_3m": (I, [P, I, I64, I64, I64, P, P, I64, P, I64, P, P, I64, P, SZ, P]),
        "ozk_s1_dgemm_unfused": (I, [P, I, I64, I64, I64, D, P, I64, P, I64, D, P, I64, P, SZ, P]),
        "ozk_s1_unfused_workspace_size": (I, [P, I, I64, I64, I64, ctypes.POINTER(SZ)]),
        "ozk_zgemm_3m": (I, [P, I, I64, I64, I64, P, P, I64, P, I64, P, P, I64, P, SZ, P]),
        "ozk_s1_split_rows": (I, [P, I, I64, I64, P, I64, P, P, P]),
        "ozk_s1_split_cols": (I, [P, I, I64, I64, P, I64, P, P, P]),
        "ozk_s1_gemm": (I, [P, I, I64, I64, I64, P, P, P, P, D, D, P, I64, P, SZ, P]),
        "ozk_s1_diagonals": (I, [P, I, I64, I64, I64, P, P, P, P]),
        "ozk_s2_split_rows": (I, [P, I, I, I64, I64, P, I64, P, P, P]),
        "ozk_s2_split_cols": (I, [P, I, I, I64, I64, P, I64, P, P, P]),
        "ozk_s2_gemm_mod": (I, [P, I, I, I64, I64, I64, P, P, P, P]),
        "ozk_s2_crt": (I, [P, I, I, I64, I64, P, P, P, P, P, P, I64, P]),
        "ozk_selector_load": (I, [P, P, SZ, P, I]),
        "ozk_select": (I, [P, D, I64, I64, I64, P, I64, P, I64, P, P, P, P, P, P]),
        "ozk_dgemm_auto": (I, [P, D, I64, I64, I64, D, P, I64, P, I64, D, P, I64, P, SZ, P, P]),
        "ozk_mlp_forward": (I, [P, P, P, I, P, P]),
        "ozk_mlp_grad": (I, [P, P, P, P, I, P, P, P]),
        "ozk_mlp_adam": (I, [P, P, P, P, P, I, ctypes.c_float, P]),
        "ozk_ref_dd": (I, [P, I64, I64, I64, P, I64, P, I64, I64, P, P, P, P, P, P]),
        "ozk_config_set": (I, [P, I, I, I, I64, I64, I64, ctypes.POINTER(OzkGemmConfig)]),
        "ozk_config_get": (I, [P, I, I, I, I64, I64, I64, ctypes.POINTER(OzkGemmConfig), ctypes.POINTER(I),
                               ctypes.POINTER(ctypes.c_float)]),
        "ozk_config_clear": (I, [P]),
        "ozk_config_save": (I, [P, ctypes.c_char_p]),
        "ozk_config_load": (I, [P, ctypes.c_char_p]),
        "ozk_tune_workspace_size": (I, [P, I, I, I, I64, I64, I64, ctypes.POINTER(SZ)]),
        "ozk_tune": (I, [P, I, I, I, I64, I64, I64, P, I64, P, I64, P, I64, P, SZ, I, ctypes.POINTER(OzkGemmConfig),
                         ctypes.POINTER(ctypes.c_float), P]),
        "ozk_batch_plan_create": (I, [P, I, I, I, I, P, ctypes.POINTER(P), ctypes.POINTER(SZ)]),
        "ozk_gemm_batched": (I, [P, P, P, SZ, P]),
        "ozk_batch_plan_destroy": (I, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


def library() -> ctypes.CDLL:
    """The loaded libozk (raises if it has not been built)."""
    return _lib()


# ------------------------------------------------------------------ helpers

def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _check(fn: str, status: int, ctx) -> None:
    if status != OZK_OK:
        arg = _lib().ozk_last_arg(ctx.handle if isinstance(ctx, Context) else ctx)
        raise OzkError(fn, status, arg)


def _need(t, name: str, dtypes, ctx, shape=None, min_numel: int = 0, dim: int = None, on_device: bool = True):
    """Raise ValueError unless t is a tensor of one of `dtypes`, of `shape`
    (when given; else of `dim` dimensions when given) and at least
    `min_numel` elements, on the CUDA device of ctx.  The checks run before
    anything is enqueued, so a wrong tensor never reaches a kernel."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError("%s must be a torch tensor, got %s" % (name, type(t).__name__))
    if not isinstance(dtypes, (tuple, list)):
        dtypes = (dtypes,)
    if t.dtype not in dtypes:
        raise ValueError("%s must have dtype %s, got %s" % (name, " or ".join(str(d) for d in dtypes), t.dtype))
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
    if shape is None and dim is not None and t.dim() != dim:
        raise ValueError("%s must be %d-dimensional, got shape %s" % (name, dim, tuple(t.shape)))
    if t.numel() < min_numel:
        raise ValueError("%s holds %d elements, at least %d are needed" % (name, t.numel(), min_numel))
    if on_device and (t.device.type != "cuda" or t.device.index != ctx.device):
        raise ValueError("%s must be on cuda:%d, got %s" % (name, ctx.device, t.device))


def _mats(ctx, dtype, A, B, C, trans_a: bool = False, trans_b: bool = False):
    """Check the operands of C = op(A) op(B) and return (M, N, K)."""
    _need(A, "A", dtype, ctx, dim=2, on_device=False)
    _need(B, "B", dtype, ctx, dim=2, on_device=False)
    M, K = (A.shape[1], A.shape[0]) if trans_a else A.shape
    Kb, N = (B.shape[1], B.shape[0]) if trans_b else B.shape
    if Kb != K:
        raise ValueError("inner dimensions differ: A gives K = %d, B gives %d" % (K, Kb))
    if C is not None:
        _need(C, "C", dtype, ctx, shape=(M, N), on_device=False)
    for t, name in ((A, "A"), (B, "B"), (C, "C")):
        if t is not None:
            _need(t, name, dtype, ctx)
    return M, N, K


def _ws(ws, ctx):
    import torch
    if ws is not None:
        _need(ws, "ws", (torch.uint8, torch.int8), ctx, dim=1)


def _ld(t) -> int:
    """Leading dimension of a row-major (unit column stride) matrix view."""
    if t.dim() == 2 and t.numel() == 0:
        return max(t.shape[1], 1)
    if t.dim() != 2 or (t.shape[1] > 1 and t.stride(1) != 1):
        raise ValueError("expected a 2-D row-major view with unit column stride")
    return max(t.stride(0), 1)


class Context:
    """An ozk context bound to one device (ozk_create / ozk_destroy).

    selector: None (no network: the auto path uses the a-priori bound),
    "default" (the parameters shipped with the package) or a path to a
    parameter file written by ``python -m paper_2606_25453_amd.selector``."""

    def __init__(self, device: int = 0, selector: Optional[str] = None):
        h = ctypes.c_void_p()
        st = _lib().ozk_create(ctypes.byref(h), device)
        if st != OZK_OK:
            raise OzkError("ozk_create", st, 0)
        self.handle = h
        self.device = device
        if selector is not None:
            from . import selector as _sel
            _sel.install(self, _sel.WEIGHTS if selector == "default" else selector)

    def close(self) -> None:
        if self.handle:
            _lib().ozk_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ozk_version() -> str:
    return _lib().ozk_version().decode()


def ozk_set_k_split(ctx: Context, k: int) -> None:
    """Testing hook: fold Scheme I K runs every k values of K (0: default)."""
    _check("ozk_set_k_split", _lib().ozk_set_k_split(ctx.handle, k), ctx)


def ozk_s1_packed_bytes(rows: int, K: int, p: int) -> int:
    return int(_lib().ozk_s1_packed_bytes(rows, K, p))


def ozk_s2_packed_bytes(rows: int, K: int, s: int, complex_planes: int = 0) -> int:
    return int(_lib().ozk_s2_packed_bytes(rows, K, s, complex_planes))


def ozk_s1_k_split(p: int) -> int:
    return int(_lib().ozk_s1_k_split(p))


def ozk_workspace_size(ctx: Context, op: int, scheme: int, M: int, N: int, K: int, p_or_s: int) -> int:
    out = ctypes.c_size_t()
    _check("ozk_workspace_size", _lib().ozk_workspace_size(ctx.handle, op, scheme, M, N, K, p_or_s,
                                                           ctypes.byref(out)), ctx)
    return int(out.value)


def _workspace(nbytes: int, device):
    import torch
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)


# --------------------------------------------------------------- whole calls

def ozk_dgemm(ctx: Context, scheme: int, p_or_s: int, A, B, C=None, alpha: float = 1.0,
              beta: float = 0.0, ws=None, stream=None):
    """C = alpha*A*B + beta*C (float64 CUDA tensors); returns C."""
    import torch
    M, N, K = _mats(ctx, torch.float64, A, B, C)
    _ws(ws, ctx)
    if C is None:
        C = torch.empty((M, N), dtype=torch.float64, device=A.device)
    if ws is None:
        ws = _workspace(ozk_workspace_size(ctx, OZK_OP_DGEMM, scheme, M, N, K, p_or_s), A.device)
    st = _lib().ozk_dgemm(ctx.handle, scheme, p_or_s, M, N, K, float(alpha), _ptr(A), _ld(A), _ptr(B), _ld(B),
                          float(beta), _ptr(C), _ld(C), _ptr(ws), ws.numel(), _stream(stream))
    _check("ozk_dgemm", st, ctx)
    return C


def ozk_dgemm_noalloc(ctx: Context, scheme: int, p_or_s: int, A, B, C=None, alpha: float = 1.0,
                      beta: float = 0.0, stream=None):
    """ozk_dgemm on the library's fixed device buffer instead of a workspace
    (nothing is allocated by the library; C is allocated here only when it
    is not given); returns C."""
    import torch
    M, N, K = _mats(ctx, torch.float64, A, B, C)
    if C is None:
        C = torch.empty((M, N), dtype=torch.float64, device=A.device)
    st = _lib().ozk_dgemm_noalloc(ctx.handle, scheme, p_or_s, M, N, K, float(alpha), _ptr(A), _ld(A), _ptr(B),
                                  _ld(B), float(beta), _ptr(C), _ld(C), _stream(stream))
    _check("ozk_dgemm_noalloc", st, ctx)
    return C


def ozk_dgemm_t(ctx: Context, scheme: int, p_or_s: int, A, B, trans_a: bool = False, trans_b: bool = False, C=None,
                alpha: float = 1.0, beta: float = 0.0, ws=None, stream=None):
    """C = alpha*op(A)*op(B) + beta*C with op(X) = X.T when its flag is set
    (A, B as stored: float64 CUDA tensors, row-major); returns C."""
    import torch
    M, N, K = _mats(ctx, torch.float64, A, B, C, bool(trans_a), bool(trans_b))
    _ws(ws, ctx)
    if C is None:
        C = torch.empty((M, N), dtype=torch.float64, device=A.device)
    if ws is None:
        ws = _workspace(ozk_workspace_size(ctx, OZK_OP_DGEMM, scheme, M, N, K, p_or_s), A.device)
    st = _lib().ozk_dgemm_t(ctx.handle, scheme, p_or_s, int(bool(trans_a)), int(bool(trans_b)), M, N, K, float(alpha),
                            _ptr(A), _ld(A), _ptr(B), _ld(B), float(beta), _ptr(C), _ld(C), _ptr(ws), ws.numel(),
                            _stream(stream))
    _check("ozk_dgemm_t", st, ctx)
    return C


def ozk_sgemm(ctx: Context, scheme: int, p_or_s: int, A, B, C=None, alpha: float = 1.0, beta: float = 0.0,
              ws=None, stream=None):
    """C = alpha*A*B + beta*C (float32 CUDA tensors) by Scheme I (p slices) or
    Scheme II (s moduli); returns C."""
    import torch
    M, N, K = _mats(ctx, torch.float32, A, B, C)
    _ws(ws, ctx)
    if C is None:
        C = torch.empty((M, N), dtype=torch.float32, device=A.device)
    if ws is None:
        ws = _workspace(ozk_workspace_size(ctx, OZK_OP_DGEMM, scheme, M, N, K, p_or_s), A.device)
    st = _lib().ozk_sgemm(ctx.handle, scheme, p_or_s, M, N, K, float(alpha), _ptr(A), _ld(A), _ptr(B), _ld(B),
                          float(beta), _ptr(C), _ld(C), _ptr(ws), ws.numel(), _stream(stream))
    _check("ozk_sgemm", st, ctx)
    return C


def ozk_s1_unfused_workspace_size(ctx: Context, p: int, M: int, N: int, K: int) -> int:
    size = ctypes.c_size_t()
    _check("ozk_s1_unfused_workspace_size",
           _lib().ozk_s1_unfused_workspace_size(ctx.handle, p, M, N, K, ctypes.byref(size)), ctx)
    return int(size.value)


def ozk_s1_dgemm_unfused(ctx: Context, p: int, A, B, C=None, alpha: float = 1.0, beta: float = 0.0, ws=None,
                         stream=None):
    """The unfused Scheme I baseline (one GEMM per slice pair, INT32 planes
    through HBM); bit-identical to ozk_dgemm(OZK_SCHEME1, p)."""
    import torch
    M, N, K = _mats(ctx, torch.float64, A, B, C)
    _ws(ws, ctx)
    if C is None:
        C = torch.empty((M, N), dtype=torch.float64, device=A.device)
    if ws is None:
        ws = _workspace(ozk_s1_unfused_workspace_size(ctx, p, M, N, K), A.device)
    st = _lib().ozk_s1_dgemm_unfused(ctx.handle, p, M, N, K, float(alpha), _ptr(A), _ld(A), _ptr(B), _ld(B),
                                     float(beta), _ptr(C), _ld(C), _ptr(ws), ws.numel(), _stream(stream))
    _check("ozk_s1_dgemm_unfused", st, ctx)
    return C


def ozk_cgemm_3m(ctx: Context, s: int, A, B, C=None, alpha: complex = 1.0, beta: complex = 0.0, ws=None,
                 stream=None):
    """C = alpha*A*B + beta*C (complex64 CUDA tensors) with Scheme II + 3M."""
    import torch
    M, N, K = _mats(ctx, torch.complex64, A, B, C)
    _ws(ws, ctx)
    if C is None:
        C = torch.empty((M, N), dtype=torch.complex64, device=A.device)
    if ws is None:
        ws = _workspace(ozk_workspace_size(ctx, OZK_OP_ZGEMM, OZK_SCHEME2, M, N, K, s), A.device)
    al = (ctypes.c_float * 2)(complex(alpha).real, complex(alpha).imag)
    be = (ctypes.c_float * 2)(complex(beta).real, complex(beta).imag)
    st = _lib().ozk_cgemm_3m(ctx.handle, s, M, N, K, ctypes.cast(al, ctypes.c_void_p), _ptr(A), _ld(A), _ptr(B),
                             _ld(B), ctypes.cast(be, ctypes.c_void_p), _ptr(C), _ld(C), _ptr(ws), ws.numel(),
                             _stream(stream))
    _check("ozk_cgemm_3m", st, ctx)
    return C


def ozk_zgemm_3m(ctx: Context, s: int, A, B, C=None, alpha: complex = 1.0, beta: complex = 0.0, ws=None,
                 stream=None):
    """C = alpha*A*B + beta*C (complex128 CUDA tensors) with Scheme II + 3M."""
    import torch
    M, N, K = _mats(ctx, torch.complex128, A, B, C)
    _ws(ws, ctx)
    if C is None:
        C = torch.empty((M, N), dtype=torch.complex128, device=A.device)
    if ws is None:
        ws = _workspace(ozk_workspace_size(ctx, OZK_OP_ZGEMM, OZK_SCHEME2, M, N, K, s), A.device)
    al = (ctypes.c_double * 2)(complex(alpha).real, complex(alpha).imag)
    be = (ctypes.c_double * 2)(complex(beta).real, complex(beta).imag)
    st = _lib().ozk_zgemm_3m(ctx.handle, s, M, N, K, ctypes.cast(al, ctypes.c_void_p), _ptr(A), _ld(A), _ptr(B),
                             _ld(B), ctypes.cast(be, ctypes.c_void_p), _ptr(C), _ld(C), _ptr(ws), ws.numel(),
                             _stream(stream))
    _check("ozk_zgemm_3m", st, ctx)
    return C


def _ld_any(t, col: bool) -> int:
    """Leading dimension of a 2-D view stored row-major (unit column stride)
    or column-major (unit row stride)."""
    if not col:
        return _ld(t)
    if t.dim() == 2 and t.numel() == 0:
        return max(t.shape[0], 1)
    if t.dim() != 2 or (t.shape[0] > 1 and t.stride(0) != 1):
        raise ValueError("expected a 2-D column-major view with unit row stride")
    return max(t.stride(1), 1)


def ozk_gemm_ex(ctx: Context, scheme: int, p_or_s: int, A, B, C=None, trans_a: bool = False, trans_b: bool = False,
                alpha=1.0, beta=0.0, ws=None, stream=None):
    """C = alpha*op(A)*op(B) + beta*C for float64, float32, complex128 or
    complex64 CUDA tensors; the storage order is that of the tensors (all
    row-major, e.g. contiguous, or all column-major, e.g. X.T of a
    contiguous matrix); op(X) = X.T when its flag is set (A, B as stored).
    Returns C (allocated column-major when the operands are and C is None)."""
    import torch
    kinds = {torch.float64: (OZK_F64, ctypes.c_double, False), torch.float32: (OZK_F32, ctypes.c_float, False),
             torch.complex128: (OZK_C128, ctypes.c_double, True), torch.complex64: (OZK_C64, ctypes.c_float, True)}
    if not isinstance(A, torch.Tensor) or A.dtype not in kinds:
        raise ValueError("A must be a float64, float32, complex128 or complex64 tensor")
    dt, real, cplx = kinds[A.dtype]
    col = A.dim() == 2 and A.shape[0] > 1 and A.stride(0) == 1 and A.shape[1] > 1 and A.stride(1) != 1
    _need(A, "A", A.dtype, ctx, dim=2)
    _need(B, "B", A.dtype, ctx, dim=2)
    M, K = (A.shape[1], A.shape[0]) if trans_a else A.shape
    Kb, N = (B.shape[1], B.shape[0]) if trans_b else B.shape
    if Kb != K:
        raise ValueError("inner dimensions differ: A gives K = %d, B gives %d" % (K, Kb))
    if C is None:
        C = torch.empty((N, M), dtype=A.dtype, device=A.device).T if col else \
            torch.empty((M, N), dtype=A.dtype, device=A.device)
    _need(C, "C", A.dtype, ctx, shape=(M, N))
    _ws(ws, ctx)
    op = OZK_OP_ZGEMM if cplx else OZK_OP_DGEMM
    if ws is None:
        mm, nn = (N, M) if col else (M, N)
        ws = _workspace(ozk_workspace_size(ctx, op, scheme, mm, nn, K, p_or_s), A.device)
    vals = (complex(alpha).real, complex(alpha).imag, complex(beta).real, complex(beta).imag)
    al = (real * 2)(vals[0], vals[1])
    be = (real * 2)(vals[2], vals[3])
    st = _lib().ozk_gemm_ex(ctx.handle, dt, OZK_COL_MAJOR if col else OZK_ROW_MAJOR, int(bool(trans_a)),
                            int(bool(trans_b)), scheme, p_or_s, M, N, K, ctypes.cast(al, ctypes.c_void_p), _ptr(A),
                            _ld_any(A, col), _ptr(B), _ld_any(B, col), ctypes.cast(be, ctypes.c_void_p), _ptr(C),
                            _ld_any(C, col), _ptr(ws), ws.numel(), _stream(stream))
    _check("ozk_gemm_ex", st, ctx)
    return C


def ozk_get_flags(ctx: Context, stream=None) -> int:
    """Wait for `stream`, then take (and clear) the context's condition flags."""
    out = ctypes.c_uint32()
    _check("ozk_get_flags", _lib().ozk_get_flags(ctx.handle, _stream(stream), ctypes.byref(out)), ctx)
    return int(out.value)


def _complex_call(name: str, dtype, real, ctx: Context, scheme: int, count: int, A, B, C, alpha, beta, ws, stream):
    import torch
    M, N, K = _mats(ctx, dtype, A, B, C)
    _ws(ws, ctx)
    if C is None:
        C = torch.empty((M, N), dtype=dtype, device=A.device)
    if ws is None:
        ws = _workspace(ozk_workspace_size(ctx, OZK_OP_ZGEMM, scheme, M, N, K, count), A.device)
    al = (real * 2)(complex(alpha).real, complex(alpha).imag)
    be = (real * 2)(complex(beta).real, complex(beta).imag)
    st = getattr(_lib(), name)(ctx.handle, scheme, count, M, N, K, ctypes.cast(al, ctypes.c_void_p), _ptr(A), _ld(A),
                               _ptr(B), _ld(B), ctypes.cast(be, ctypes.c_void_p), _ptr(C), _ld(C), _ptr(ws),
                               ws.numel(), _stream(stream))
    _check(name, st, ctx)
    return C


def ozk_zgemm(ctx: Context, scheme: int, p_or_s: int, A, B, C=None, alpha: complex = 1.0, beta: complex = 0.0,
              ws=None, stream=None):
    """C = alpha*A*B + beta*C (complex128 CUDA tensors) by Scheme I with 4M
    (p slices) or Scheme II with 3M (s moduli); returns C."""
    import torch
    return _complex_call("ozk_zgemm", torch.complex128, ctypes.c_double, ctx, scheme, p_or_s, A, B, C, alpha, beta,
                         ws, stream)


def ozk_cgemm(ctx: Context, scheme: int, p_or_s: int, A, B, C=None, alpha: complex = 1.0, beta: complex = 0.0,
              ws=None, stream=None):
    """ozk_zgemm in complex64 (binary32 parts in and out); returns C."""
    import torch
    return _complex_call("ozk_cgemm", torch.complex64, ctypes.c_float, ctx, scheme, p_or_s, A, B, C, alpha, beta,
                         ws, stream)


def ozk_s2_unfused_workspace_size(ctx: Context, s: int, complex_planes: int, M: int, N: int, K: int) -> int:
    out = ctypes.c_size_t()
    _check("ozk_s2_unfused_workspace_size",
           _lib().ozk_s2_unfused_workspace_size(ctx.handle, s, complex_planes, M, N, K, ctypes.byref(out)), ctx)
    return int(out.value)


def ozk_s2_gemm_unfused(ctx: Context, s: int, A, B, C=None, alpha: complex = 1.0, beta: complex = 0.0, ws=None,
                        stream=None):
    """The unfused Scheme II baseline (INT32 planes through HBM): float64
    operands give the real product, complex128 ones the 3M product; returns C."""
    import torch
    cplx = A.dtype == torch.complex128
    dtype = torch.complex128 if cplx else torch.float64
    M, N, K = _mats(ctx, dtype, A, B, C)
    _ws(ws, ctx)
    if C is None:
        C = torch.empty((M, N), dtype=dtype, device=A.device)
    if ws is None:
        ws = _workspace(ozk_s2_unfused_workspace_size(ctx, s, int(cplx), M, N, K), A.device)
    al = (ctypes.c_double * 2)(complex(alpha).real, complex(alpha).imag)
    be = (ctypes.c_double * 2)(complex(beta).real, complex(beta).imag)
    st = _lib().ozk_s2_gemm_unfused(ctx.handle, s, int(cplx), M, N, K, ctypes.cast(al, ctypes.c_void_p), _ptr(A),
                                    _ld(A), _ptr(B), _ld(B), ctypes.cast(be, ctypes.c_void_p), _ptr(C), _ld(C),
                                    _ptr(ws), ws.numel(), _stream(stream))
    _check("ozk_s2_gemm_unfused", st, ctx)
    return C


def ozk_zgemm_auto(ctx: Context, tol: float, A, B, C=None, alpha: complex = 1.0, beta: complex = 0.0, ws=None,
                   info=None, stream=None):
    """ZGEMM (complex128 CUDA tensors) by 3M with the modulus count chosen on
    the device for the tolerance; returns (C, info)."""
    import torch
    M, N, K = _mats(ctx, torch.complex128, A, B, C)
    _ws(ws, ctx)
    if info is not None:
        _need(info, "info", torch.int32, ctx, min_numel=OZK_SELECTOR_INFO)
    if C is None:
        C = torch.empty((M, N), dtype=torch.complex128, device=A.device)
    if ws is None:
        ws = _workspace(ozk_workspace_size(ctx, OZK_OP_ZGEMM, OZK_SCHEME2, M, N, K, 0), A.device)
    if info is None:
        info = torch.empty(OZK_SELECTOR_INFO, dtype=torch.int32, device=A.device)
    al = (ctypes.c_double * 2)(complex(alpha).real, complex(alpha).imag)
    be = (ctypes.c_double * 2)(complex(beta).real, complex(beta).imag)
    st = _lib().ozk_zgemm_auto(ctx.handle, float(tol), M, N, K, ctypes.cast(al, ctypes.c_void_p), _ptr(A), _ld(A),
                               _ptr(B), _ld(B), ctypes.cast(be, ctypes.c_void_p), _ptr(C), _ld(C), _ptr(ws),
                               ws.numel(), _ptr(info), _stream(stream))
    _check("ozk_zgemm_auto", st, ctx)
    return C, info


# ---------------------------------------------------------- Scheme I steps

def ozk_s1_split_rows(ctx: Context, p: int, X, e=None, packed=None, stream=None):
    """Row exponents and packed slices of a row operand; returns (e, packed)."""
    import torch
    _need(X, "X", torch.float64, ctx, dim=2)
    rows, K = X.shape
    if e is not None:
        _need(e, "e", torch.int32, ctx, min_numel=rows)
    if packed is not None:
        _need(packed, "packed", torch.int8, ctx, min_numel=ozk_s1_packed_bytes(rows, K, p))
    if e is None:
        e = torch.empty(max(rows, 1), dtype=torch.int32, device=X.device)
    if packed is None:
        packed = torch.empty(max(ozk_s1_packed_bytes(rows, K, p), 1), dtype=torch.int8, device=X.device)
    st = _lib().ozk_s1_split_rows(ctx.handle, p, rows, K, _ptr(X), _ld(X), _ptr(e), _ptr(packed), _stream(stream))
    _check("ozk_s1_split_rows", st, ctx)
    return e, packed


def ozk_s1_split_cols(ctx: Context, p: int, X, f=None, packed=None, stream=None):
    """Column exponents and packed (transposed) slices of a column operand."""
    import torch
    _need(X, "X", torch.float64, ctx, dim=2)
    K, cols = X.shape
    if f is not None:
        _need(f, "f", torch.int32, ctx, min_numel=cols)
    if packed is not None:
        _need(packed, "packed", torch.int8, ctx, min_numel=ozk_s1_packed_bytes(cols, K, p))
    if f is None:
        f = torch.empty(max(cols, 1), dtype=torch.int32, device=X.device)
    if packed is None:
        packed = torch.empty(max(ozk_s1_packed_bytes(cols, K, p), 1), dtype=torch.int8, device=X.device)
    st = _lib().ozk_s1_split_cols(ctx.handle, p, K, cols, _ptr(X), _ld(X), _ptr(f), _ptr(packed), _stream(stream))
    _check("ozk_s1_split_cols", st, ctx)
    return f, packed


def ozk_s1_gemm(ctx: Context, p: int, M: int, N: int, K: int, packedA, e, packedB, f, C, alpha: float = 1.0,
                beta: float = 0.0, ws=None, stream=None):
    import torch
    _need(packedA, "packedA", torch.int8, ctx, min_numel=ozk_s1_packed_bytes(M, K, p))
    _need(packedB, "packedB", torch.int8, ctx, min_numel=ozk_s1_packed_bytes(N, K, p))
    _need(e, "e", torch.int32, ctx, min_numel=M)
    _need(f, "f", torch.int32, ctx, min_numel=N)
    _need(C, "C", torch.float64, ctx, shape=(M, N))
    _ws(ws, ctx)
    st = _lib().ozk_s1_gemm(ctx.handle, p, M, N, K, _ptr(packedA), _ptr(e), _ptr(packedB), _ptr(f), float(alpha),
                            float(beta), _ptr(C), _ld(C), _ptr(ws), 0 if ws is None else ws.numel(),
                            _stream(stream))
    _check("ozk_s1_gemm", st, ctx)
    return C


def ozk_s1_diagonals(ctx: Context, p: int, M: int, N: int, K: int, packedA, packedB, Cd=None, stream=None):
    """Raw INT32 diagonals [p][M][N] of the fused kernel."""
    import torch
    _need(packedA, "packedA", torch.int8, ctx, min_numel=ozk_s1_packed_bytes(M, K, p))
    _need(packedB, "packedB", torch.int8, ctx, min_numel=ozk_s1_packed_bytes(N, K, p))
    if Cd is not None:
        _need(Cd, "Cd", torch.int32, ctx, shape=(p, M, N))
    if Cd is None:
        Cd = torch.empty((p, M, N), dtype=torch.int32, device=packedA.device)
    st = _lib().ozk_s1_diagonals(ctx.handle, p, M, N, K, _ptr(packedA), _ptr(packedB), _ptr(Cd), _stream(stream))
    _check("ozk_s1_diagonals", st, ctx)
    return Cd


# --------------------------------------------------------- Scheme II steps

def ozk_s2_split_rows(ctx: Context, s: int, X, complex_planes: int = 0, sigma=None, packed=None, stream=None):
    import torch
    _need(X, "X", torch.complex128 if complex_planes else torch.float64, ctx, dim=2)
    rows, K = X.shape
    if sigma is not None:
        _need(sigma, "sigma", torch.int32, ctx, min_numel=rows)
    if packed is not None:
        _need(packed, "packed", torch.int8, ctx, min_numel=ozk_s2_packed_bytes(rows, K, s, complex_planes))
    if sigma is None:
        sigma = torch.empty(max(rows, 1), dtype=torch.int32, device=X.device)
    if packed is None:
        packed = torch.empty(max(ozk_s2_packed_bytes(rows, K, s, complex_planes), 1), dtype=torch.int8,
                             device=X.device)
    st = _lib().ozk_s2_split_rows(ctx.handle, s, complex_planes, rows, K, _ptr(X), _ld(X), _ptr(sigma),
                                  _ptr(packed), _stream(stream))
    _check("ozk_s2_split_rows", st, ctx)
    return sigma, packed


def ozk_s2_split_cols(ctx: Context, s: int, X, complex_planes: int = 0, tau=None, packed=None, stream=None):
    import torch
    _need(X, "X", torch.complex128 if complex_planes else torch.float64, ctx, dim=2)
    K, cols = X.shape
    if tau is not None:
        _need(tau, "tau", torch.int32, ctx, min_numel=cols)
    if packed is not None:
        _need(packed, "packed", torch.int8, ctx, min_numel=ozk_s2_packed_bytes(cols, K, s, complex_planes))
    if tau is None:
        tau = torch.empty(max(cols, 1), dtype=torch.int32, device=X.device)
    if packed is None:
        packed = torch.empty(max(ozk_s2_packed_bytes(cols, K, s, complex_planes), 1), dtype=torch.int8,
                             device=X.device)
    st = _lib().ozk_s2_split_cols(ctx.handle, s, complex_planes, K, cols, _ptr(X), _ld(X), _ptr(tau),
                                  _ptr(packed), _stream(stream))
    _check("ozk_s2_split_cols", st, ctx)
    return tau, packed


def ozk_s2_gemm_mod(ctx: Context, s: int, M: int, N: int, K: int, packedA, packedB, complex_planes: int = 0,
                    Cres=None, stream=None):
    import torch
    _need(packedA, "packedA", torch.int8, ctx, min_numel=ozk_s2_packed_bytes(M, K, s, complex_planes))
    _need(packedB, "packedB", torch.int8, ctx, min_numel=ozk_s2_packed_bytes(N, K, s, complex_planes))
    if Cres is not None:
        _need(Cres, "Cres", torch.int8, ctx, shape=(s * (2 if complex_planes else 1), M, N))
    if Cres is None:
        Cres = torch.empty((s * (2 if complex_planes else 1), M, N), dtype=torch.int8, device=packedA.device)
    st = _lib().ozk_s2_gemm_mod(ctx.handle, s, complex_planes, M, N, K, _ptr(packedA), _ptr(packedB), _ptr(Cres),
                                _stream(stream))
    _check("ozk_s2_gemm_mod", st, ctx)
    return Cres


def ozk_s2_crt(ctx: Context, s: int, M: int, N: int, Cres, sigma, tau, C, alpha=1.0, beta=0.0,
               complex_planes: int = 0, stream=None):
    import torch
    _need(Cres, "Cres", torch.int8, ctx, shape=(s * (2 if complex_planes else 1), M, N))
    _need(sigma, "sigma", torch.int32, ctx, min_numel=M)
    _need(tau, "tau", torch.int32, ctx, min_numel=N)
    _need(C, "C", torch.complex128 if complex_planes else torch.float64, ctx, shape=(M, N))
    al = (ctypes.c_double * 2)(complex(alpha).real, complex(alpha).imag)
    be = (ctypes.c_double * 2)(complex(beta).real, complex(beta).imag)
    st = _lib().ozk_s2_crt(ctx.handle, s, complex_planes, M, N, _ptr(Cres), _ptr(sigma), _ptr(tau),
                           ctypes.cast(al, ctypes.c_void_p), ctypes.cast(be, ctypes.c_void_p), _ptr(C), _ld(C),
                           _stream(stream))
    _check("ozk_s2_crt", st, ctx)
    return C


# ----------------------------------------------------------- layout helpers

def unpack_s1(packed, rows: int, K: int, p: int):
    """View a Scheme I packed operand (a torch int8 tensor) as [p][rows][K]
    (drops the padding); a pure reshape of the documented layout."""
    Rp = (rows + OZK_ROW_ALIGN - 1) // OZK_ROW_ALIGN * OZK_ROW_ALIGN
    Kp = (K + OZK_K_CHUNK - 1) // OZK_K_CHUNK * OZK_K_CHUNK
    v = packed[: Rp * Kp * p].reshape(Kp // OZK_K_CHUNK, p, Rp, OZK_K_CHUNK)
    v = v.permute(1, 2, 0, 3).reshape(p, Rp, Kp)
    return v[:, :rows, :K]


# ------------------------------------------------------------------ batches

class OzkGemmDesc(ctypes.Structure):
    """ozk_gemm_desc of include/ozk.h."""
    _fields_ = [("M", ctypes.c_int64), ("N", ctypes.c_int64), ("K", ctypes.c_int64),
                ("A", ctypes.c_void_p), ("lda", ctypes.c_int64),
                ("B", ctypes.c_void_p), ("ldb", ctypes.c_int64),
                ("C", ctypes.c_void_p), ("ldc", ctypes.c_int64),
                ("alpha", ctypes.c_double * 2), ("beta", ctypes.c_double * 2)]


def ozk_batch_plan_create(ctx: Context, op: int, scheme: int, p_or_s: int, descs):
    """Plan a batch from a sequence of OzkGemmDesc; returns (plan, ws_bytes)."""
    arr = (OzkGemmDesc * max(len(descs), 1))(*descs)
    plan = ctypes.c_void_p()
    ws = ctypes.c_size_t()
    st = _lib().ozk_batch_plan_create(ctx.handle, op, scheme, p_or_s, len(descs), ctypes.cast(arr, ctypes.c_void_p),
                                      ctypes.byref(plan), ctypes.byref(ws))
    _check("ozk_batch_plan_create", st, ctx)
    return plan, int(ws.value)


def ozk_gemm_batched(ctx: Context, plan, ws, stream=None) -> None:
    st = _lib().ozk_gemm_batched(ctx.handle, plan, _ptr(ws), ws.numel(), _stream(stream))
    _check("ozk_gemm_batched", st, ctx)


def ozk_batch_plan_destroy(plan) -> None:
    _lib().ozk_batch_plan_destroy(plan)


class BatchPlan:
    """A planned batch over (A, B, C) CUDA tensors (float64 for DGEMM,
    complex128 for ZGEMM) that owns its workspace; run() enqueues the whole
    batch on a stream (graph-capturable)."""

    def __init__(self, ctx: Context, op: int, scheme: int, p_or_s: int, problems, alpha=1.0, beta=0.0):
        import torch
        self.ctx = ctx
        self.keep = list(problems)  # the plan keeps raw pointers to these tensors
        al, be = complex(alpha), complex(beta)
        dtype = torch.complex128 if op == OZK_OP_ZGEMM else torch.float64
        for i, (A, B, C) in enumerate(self.keep):
            try:
                _mats(ctx, dtype, A, B, C)
            except ValueError as err:
                raise ValueError("problem %d: %s" % (i, err)) from None
        descs = []
        for A, B, C in self.keep:
            d = OzkGemmDesc()
            d.M, d.K = A.shape
            d.N = B.shape[1]
            d.A, d.lda = _ptr(A), _ld(A)
            d.B, d.ldb = _ptr(B), _ld(B)
            d.C, d.ldc = _ptr(C), _ld(C)
            d.alpha[0], d.alpha[1] = al.real, al.imag
            d.beta[0], d.beta[1] = be.real, be.imag
            descs.append(d)
        self.plan, nbytes = ozk_batch_plan_create(ctx, op, scheme, p_or_s, descs)
        dev = self.keep[0][0].device if self.keep else torch.device("cuda:0")
        self.ws = _workspace(nbytes, dev)

    def run(self, stream=None) -> None:
        ozk_gemm_batched(self.ctx, self.plan, self.ws, stream)

    def tiles(self):
        """1 for each problem on the 128 x 128 tile, 0 on 64 x 64."""
        out = (ctypes.c_int32 * max(len(self.keep), 1))()
        st = _lib().ozk_batch_plan_tiles(self.plan, len(self.keep), ctypes.cast(out, ctypes.c_void_p))
        if st != OZK_OK:
            raise OzkError("ozk_batch_plan_tiles", st, 0)
        return [int(out[i]) for i in range(len(self.keep))]

    def tune(self, reps: int = 3, stream=None) -> None:
        """ozk_tune_batch: choose each size class's tile on these problems
        (synchronises) and leave the batch computed."""
        st = _lib().ozk_tune_batch(self.ctx.handle, self.plan, _ptr(self.ws), self.ws.numel(), int(reps),
                                   _stream(stream))
        _check("ozk_tune_batch", st, self.ctx)

    def close(self) -> None:
        if self.plan:
            ozk_batch_plan_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- autotuner

def ozk_config_set(ctx: Context, op: int, scheme: int, p_or_s: int, M: int, N: int, K: int, config) -> None:
    """Store a configuration (OzkGemmConfig or a 4-tuple) for the size class of (M, N, K)."""
    cfg = config if isinstance(config, OzkGemmConfig) else OzkGemmConfig(*config)
    _check("ozk_config_set", _lib().ozk_config_set(ctx.handle, op, scheme, p_or_s, M, N, K, ctypes.byref(cfg)), ctx)


def ozk_config_get(ctx: Context, op: int, scheme: int, p_or_s: int, M: int, N: int, K: int):
    """(config tuple, found, tuned ms) for the size class of (M, N, K)."""
    cfg = OzkGemmConfig()
    found = ctypes.c_int()
    ms = ctypes.c_float()
    _check("ozk_config_get", _lib().ozk_config_get(ctx.handle, op, scheme, p_or_s, M, N, K, ctypes.byref(cfg),
                                                   ctypes.byref(found), ctypes.byref(ms)), ctx)
    return cfg.as_tuple(), bool(found.value), float(ms.value)


def ozk_config_clear(ctx: Context) -> None:
    _check("ozk_config_clear", _lib().ozk_config_clear(ctx.handle), ctx)


def ozk_config_save(ctx: Context, path: str) -> None:
    _check("ozk_config_save", _lib().ozk_config_save(ctx.handle, os.fsencode(path)), ctx)


def ozk_config_load(ctx: Context, path: str) -> None:
    _check("ozk_config_load", _lib().ozk_config_load(ctx.handle, os.fsencode(path)), ctx)


def ozk_tune_workspace_size(ctx: Context, op: int, scheme: int, p_or_s: int, M: int, N: int, K: int) -> int:
    out = ctypes.c_size_t()
    _check("ozk_tune_workspace_size", _lib().ozk_tune_workspace_size(ctx.handle, op, scheme, p_or_s, M, N, K,
                                                                     ctypes.byref(out)), ctx)
    return int(out.value)


def ozk_tune(ctx: Context, op: int, scheme: int, p_or_s: int, A, B, C=None, reps: int = 3, ws=None, stream=None):
    """Tune the size class of A B (float64 or complex128 CUDA tensors); returns
    (C = A B, best config tuple, best ms)."""
    import torch
    M, N, K = _mats(ctx, torch.complex128 if op == OZK_OP_ZGEMM else torch.float64, A, B, C)
    _ws(ws, ctx)
    if C is None:
        C = torch.empty((M, N), dtype=A.dtype, device=A.device)
    if ws is None:
        ws = _workspace(ozk_tune_workspace_size(ctx, op, scheme, p_or_s, M, N, K), A.device)
    best = OzkGemmConfig()
    ms = ctypes.c_float()
    st = _lib().ozk_tune(ctx.handle, op, scheme, p_or_s, M, N, K, _ptr(A), _ld(A), _ptr(B), _ld(B), _ptr(C), _ld(C),
                         _ptr(ws), ws.numel(), reps, ctypes.byref(best), ctypes.byref(ms), _stream(stream))
    _check("ozk_tune", st, ctx)
    return C, best.as_tuple(), float(ms.value)


# ------------------------------------------------------- slice-count selector

def ozk_select(ctx: Context, tol: float, A, B, stream=None):
    """Device statistics and decision for A B: (e, f, counters, info, features)
    as device tensors; info = [p (0 with Scheme II), p_net, p_bound,
    out_of_range, scheme, s (0 with Scheme I), s_bound, 0]."""
    import torch
    M, N, K = _mats(ctx, torch.float64, A, B, None)
    e = torch.empty(max(M, 1), dtype=torch.int32, device=A.device)
    f = torch.empty(max(N, 1), dtype=torch.int32, device=A.device)
    cnt = torch.empty(OZK_SELECTOR_COUNTERS, dtype=torch.int32, device=A.device)
    info = torch.empty(OZK_SELECTOR_INFO, dtype=torch.int32, device=A.device)
    feat = torch.empty(34, dtype=torch.float32, device=A.device)
    st = _lib().ozk_select(ctx.handle, float(tol), M, N, K, _ptr(A), _ld(A), _ptr(B), _ld(B), _ptr(e), _ptr(f),
                           _ptr(cnt), _ptr(info), _ptr(feat), _stream(stream))
    _check("ozk_select", st, ctx)
    return e[:M], f[:N], cnt, info, feat


def ozk_dgemm_auto(ctx: Context, tol: float, A, B, C=None, alpha: float = 1.0, beta: float = 0.0, ws=None,
                   info=None, stream=None):
    """DGEMM with the scheme and slice or modulus count chosen on the device
    for the componentwise tolerance tol; returns (C, info) with info the
    device int32[8] decision (see ozk_select)."""
    import torch
    M, N, K = _mats(ctx, torch.float64, A, B, C)
    _ws(ws, ctx)
    if info is not None:
        _need(info, "info", torch.int32, ctx, min_numel=OZK_SELECTOR_INFO)
    if C is None:
        C = torch.empty((M, N), dtype=torch.float64, device=A.device)
    if ws is None:
        ws = _workspace(ozk_workspace_size(ctx, OZK_OP_DGEMM, OZK_SCHEME1, M, N, K, 0), A.device)
    if info is None:
        info = torch.empty(OZK_SELECTOR_INFO, dtype=torch.int32, device=A.device)
    st = _lib().ozk_dgemm_auto(ctx.handle, float(tol), M, N, K, float(alpha), _ptr(A), _ld(A), _ptr(B), _ld(B),
                               float(beta), _ptr(C), _ld(C), _ptr(ws), ws.numel(), _ptr(info), _stream(stream))
    _check("ozk_dgemm_auto", st, ctx)
    return C, info
