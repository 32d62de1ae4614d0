"""Plain CPU oracle for Ozaki-scheme emulated FP64 / complex128 GEMM.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The emulation library
never imports it, and it imports nothing from the library: the two share no
code, tables or helpers.  Inputs come from the caller (the seeded generators
live in their own module, ``synth``).

What it computes (section / equation numbers are the paper's):

* ``gemm_naive``, ``gemm_dd``, ``zgemm_dd`` -- reference products (plain FP64
  with fma; double-double with error-free transformations).
* Scheme I (Sec. II-C.1, Eqs. 1-3; Sec. III, Alg. 1): row/column power-of-two
  scales, 8-bit slices as balanced signed base-256 digits of the rounded
  fixed-point value (8p-2 bits in all; every slice is a signed INT8), the p
  triangular slice-pair diagonals, and the exact shift-reduce + one correctly
  rounded scaling.
  Implemented in ``ozk_oracle.c`` (built with gcc, OpenMP) and wrapped here.
* Scheme II (Sec. II-C.2, Eqs. 4-8) and its 3M complex form (Sec. IV-B,
  Eq. 16): in ``scheme2`` (numpy integer products, Python big-integer CRT).
* Error metrics and the analytic bound used as the selector's fallback:
  in ``metrics``.

Readings of points the paper leaves open are listed beside each function.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ozk_oracle.c")
_LIB = os.path.join(_HERE, "_ozk_oracle.so")

ZERO_EXP = -100000
NONFINITE_EXP = 100000

_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (plain C, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    D = ctypes.c_double
    I = ctypes.c_int
    sig = {
        "orc_gemm_naive": (None, [I64, I64, I64, P, P, P]),
        "orc_gemm_dd": (None, [I64, I64, I64, P, P, P, P]),
        "orc_zgemm_dd": (None, [I64, I64, I64, P, P, P, P]),
        "orc_expo": (I, [D]),
        "orc_s1_row_exponents": (None, [I64, I64, P, P]),
        "orc_s1_col_exponents": (None, [I64, I64, P, P]),
        "orc_s1_digits_a": (None, [I64, I64, P, P, I, P]),
        "orc_s1_digits_b": (None, [I64, I64, P, P, I, P]),
        "orc_s1_diagonals": (None, [I64, I64, I64, I, P, P, P]),
        "orc_s1_reconstruct": (None, [I64, I64, I, P, P, P, D, D, P]),
        "orc_s1_z": (None, [I64, I64, I, P, P, P]),
        "orc_s1_dgemm": (I, [I64, I64, I64, I, D, P, P, D, P]),
        "orc_s1_entries": (None, [I64, I64, I64, I, D, P, P, P, P, I64, P, P, P, D, P]),
        "orc_round_scaled_parts": (D, [I64, I64, I64]),
        "orc_round_scaled_f32_parts": (ctypes.c_float, [I64, I64, I64]),
        "orc_s1_sgemm": (I, [I64, I64, I64, I, ctypes.c_float, P, P, ctypes.c_float, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------- references

def gemm_naive(A, B) -> np.ndarray:
    """Plain FP64 triple loop, k ascending, one fma per term."""
    A, B = _f64(A), _f64(B)
    M, K = A.shape
    N = B.shape[1]
    C = np.empty((M, N), np.float64)
    _load().orc_gemm_naive(M, N, K, _p(A), _p(B), _p(C))
    return C


def gemm_dd(A, B):
    """Double-double product: returns (hi, lo) with hi + lo ~ A B to ~2^-104."""
    A, B = _f64(A), _f64(B)
    M, K = A.shape
    N = B.shape[1]
    hi = np.empty((M, N), np.float64)
    lo = np.empty((M, N), np.float64)
    _load().orc_gemm_dd(M, N, K, _p(A), _p(B), _p(hi), _p(lo))
    return hi, lo


def zgemm_dd(A, B):
    """Complex double-double product; returns (hi, lo) complex128 arrays."""
    A = np.ascontiguousarray(A, dtype=np.complex128)
    B = np.ascontiguousarray(B, dtype=np.complex128)
    M, K = A.shape
    N = B.shape[1]
    hi = np.empty((M, N), np.complex128)
    lo = np.empty((M, N), np.complex128)
    _load().orc_zgemm_dd(M, N, K, _p(A), _p(B), _p(hi), _p(lo))
    return hi, lo


# ------------------------------------------------------------------ Scheme I

def expo(x: float) -> int:
    """frexp exponent e of a finite nonzero x: 2^(e-1) <= |x| < 2^e."""
    return int(_load().orc_expo(float(x)))


def s1_row_exponents(A) -> np.ndarray:
    """e_i = max_k expo(a_ik) over nonzero entries (row scale mu_i = 2^e_i)."""
    A = _f64(A)
    M, K = A.shape
    e = np.empty(M, np.int32)
    _load().orc_s1_row_exponents(M, K, _p(A), _p(e))
    return e


def s1_col_exponents(B) -> np.ndarray:
    """f_j = max_k expo(b_kj) over nonzero entries (column scale nu_j)."""
    B = _f64(B)
    K, N = B.shape
    f = np.empty(N, np.int32)
    _load().orc_s1_col_exponents(K, N, _p(B), _p(f))
    return f


def s1_digits_a(A, e, p: int) -> np.ndarray:
    """Slices of A as int8 [p][M][K] (Eq. 1): with X = floor(a 2^(8p-2-e_i) + 1/2),
    the balanced base-256 digits of X (|d_0| <= 64, d_t in [-128, 127]), so
    that a 2^-e_i = sum_t d_t 2^(-6-8t) to within 2^-(8p-1)."""
    A = _f64(A)
    M, K = A.shape
    D = np.empty((p, M, K), np.int8)
    e = np.ascontiguousarray(e, np.int32)
    _load().orc_s1_digits_a(M, K, _p(A), _p(e), p, _p(D))
    return D


def s1_digits_b(B, f, p: int) -> np.ndarray:
    """Slices of B as int8 [p][K][N], same format along columns."""
    B = _f64(B)
    K, N = B.shape
    E = np.empty((p, K, N), np.int8)
    f = np.ascontiguousarray(f, np.int32)
    _load().orc_s1_digits_b(K, N, _p(B), _p(f), p, _p(E))
    return E


def s1_diagonals(D, E) -> np.ndarray:
    """Eq. 2: Cd[d] = sum_{t<=d} D_t E_{d-t}, exact int64 [p][M][N]."""
    D = np.ascontiguousarray(D, np.int8)
    E = np.ascontiguousarray(E, np.int8)
    p, M, K = D.shape
    N = E.shape[2]
    Cd = np.empty((p, M, N), np.int64)
    _load().orc_s1_diagonals(M, N, K, p, _p(D), _p(E), _p(Cd))
    return Cd


def s1_z(Cd) -> list:
    """Exact shift-reduce integer Z = sum_d 2^(8(p-1-d)) Cd[d], as Python ints."""
    Cd = np.ascontiguousarray(Cd, np.int64)
    p, M, N = Cd.shape
    lo = np.empty(M * N, np.int64)
    hi = np.empty(M * N, np.int64)
    _load().orc_s1_z(M, N, p, _p(Cd), _p(lo), _p(hi))
    return [(int(h) << 64) + (int(l) & ((1 << 64) - 1)) for l, h in zip(lo, hi)]


def s1_reconstruct(Cd, e, f, alpha=1.0, beta=0.0, C=None) -> np.ndarray:
    """Eq. 3 made exact: RN(Z 2^(e_i+f_j-12-8(p-1))), then alpha/beta."""
    Cd = np.ascontiguousarray(Cd, np.int64)
    p, M, N = Cd.shape
    out = np.zeros((M, N), np.float64) if C is None else _f64(C).copy()
    e = np.ascontiguousarray(e, np.int32)
    f = np.ascontiguousarray(f, np.int32)
    _load().orc_s1_reconstruct(M, N, p, _p(Cd), _p(e), _p(f), float(alpha), float(beta), _p(out))
    return out


def s1_dgemm(A, B, p: int, alpha=1.0, beta=0.0, C=None) -> np.ndarray:
    """Whole Scheme I DGEMM: C = alpha * emu(A B) + beta * C."""
    A, B = _f64(A), _f64(B)
    M, K = A.shape
    N = B.shape[1]
    out = np.zeros((M, N), np.float64) if C is None else _f64(C).copy()
    rc = _load().orc_s1_dgemm(M, N, K, p, float(alpha), _p(A), _p(B), float(beta), _p(out))
    if rc != 0:
        raise ValueError("orc_s1_dgemm failed (%d)" % rc)
    return out


def s1_entries(A, B, p: int, rows, cols, alpha=1.0, beta=0.0, cin=None) -> np.ndarray:
    """Scheme I outputs (rows[s], cols[s]) only, computed one by one."""
    A, B = _f64(A), _f64(B)
    M, K = A.shape
    N = B.shape[1]
    rows = np.ascontiguousarray(rows, np.int64)
    cols = np.ascontiguousarray(cols, np.int64)
    n = rows.size
    e = s1_row_exponents(A)
    f = s1_col_exponents(B)
    cin = np.zeros(n, np.float64) if cin is None else _f64(cin)
    out = np.empty(n, np.float64)
    _load().orc_s1_entries(M, N, K, p, float(alpha), _p(A), _p(B), _p(e), _p(f), n,
                           _p(rows), _p(cols), _p(cin), float(beta), _p(out))
    return out


def round_scaled(Z: int, E: int) -> float:
    """The C oracle's RN(Z 2^E) for |Z| < 2^127 (exposed for pinning)."""
    lo = Z & ((1 << 64) - 1)
    hi = Z >> 64
    if lo >= 1 << 63:
        lo -= 1 << 64
    return float(_load().orc_round_scaled_parts(lo, hi, E))


def s1_scale_exponent(e: int, f: int, p: int) -> int:
    """Exponent E with emulated (A B)_ij = Z_ij 2^E (E = e_i + f_j - 12 - 8(p-1))."""
    return int(e) + int(f) - 12 - 8 * (p - 1)


def k_split_s1(p: int) -> int:
    """Longest K run (a multiple of 32) over which no INT32 diagonal can
    overflow: |d_0| <= 64 and |d_t| <= 128 bound diagonal d by
    max(2^12, d 2^14) per k."""
    per_k = max(2 ** 12, (p - 1) * 2 ** 14)
    return ((2 ** 31 - 1) // per_k) // 32 * 32


from . import scheme2, metrics, selector  # noqa: E402,F401


def round_scaled_f32(Z: int, E: int) -> np.float32:
    """The C oracle's RN(Z 2^E) to binary32 for |Z| < 2^127 (exposed for pinning)."""
    lo = Z & ((1 << 64) - 1)
    hi = Z >> 64
    if lo >= 1 << 63:
        lo -= 1 << 64
    return np.float32(_load().orc_round_scaled_f32_parts(lo, hi, E))


def s1_sgemm(A, B, p: int, alpha=1.0, beta=0.0, C=None) -> np.ndarray:
    """Whole Scheme I SGEMM on binary32 operands: the binary64 pipeline on the
    exactly widened operands, one rounding of Z 2^E to binary32, then
    C = alpha * h + beta * C in binary32."""
    A = np.ascontiguousarray(A, np.float32)
    B = np.ascontiguousarray(B, np.float32)
    M, K = A.shape
    N = B.shape[1]
    out = np.zeros((M, N), np.float32) if C is None else np.ascontiguousarray(C, np.float32).copy()
    rc = _load().orc_s1_sgemm(M, N, K, p, float(alpha), _p(A), _p(B), float(beta), _p(out))
    if rc != 0:
        raise ValueError("orc_s1_sgemm failed (%d)" % rc)
    return out


# ------------------------------------------------- Scheme I complex (4M)

def s1_complex_embed(A, B):
    """The real matrices whose product holds the four real products of the
    4M complex product (Sec. IV-B): A' = [Re A, Im A] (M x 2K) and B'' (2K x
    2N) with, for k < K,
        B''[k, 2j] = Re B[k, j],      B''[k, 2j+1] = Im B[k, j],
        B''[K+k, 2j] = -Im B[k, j],   B''[K+k, 2j+1] = Re B[k, j],
    so that (A' B'')[i, 2j] = Re(A B)[i, j] and (A' B'')[i, 2j+1] = Im(A B)[i, j]
    (Re = Ar Br - Ai Bi, Im = Ar Bi + Ai Br).  Row i of A' holds both parts of
    row i of A, so its Scheme I exponent is shared by them; columns 2j and
    2j+1 of B'' hold the same magnitudes, so they share one exponent."""
    A = np.asarray(A)
    B = np.asarray(B)
    real = np.float32 if A.dtype == np.complex64 else np.float64
    M, K = A.shape
    N = B.shape[1]
    A2 = np.concatenate([A.real, A.imag], axis=1).astype(real)
    B2 = np.empty((2 * K, 2 * N), real)
    B2[:K, 0::2] = B.real
    B2[:K, 1::2] = B.imag
    B2[K:, 0::2] = -B.imag
    B2[K:, 1::2] = B.real
    return np.ascontiguousarray(A2), B2


def s1_zgemm(A, B, p: int, alpha=1.0, beta=0.0, C=None) -> np.ndarray:
    """Scheme I ZGEMM by 4M: Scheme I (p slices) on the embedded real
    matrices, whose exact integer products are the four real products with
    the subtraction and addition of 4M done before the one rounding of each
    part; then the complex alpha/beta update of zaxpby."""
    from .scheme2 import zaxpby
    A2, B2 = s1_complex_embed(np.asarray(A, np.complex128), np.asarray(B, np.complex128))
    H2 = s1_dgemm(A2, B2, p)
    H = H2[:, 0::2] + 1j * H2[:, 1::2]
    return zaxpby(alpha, H, beta, C)


def s1_cgemm(A, B, p: int, alpha=1.0, beta=0.0, C=None) -> np.ndarray:
    """Scheme I CGEMM (complex64 in and out) by 4M: the embedded binary32
    matrices through the Scheme I SGEMM steps (one rounding of each part to
    binary32), then the complex alpha/beta update in binary32."""
    from .scheme2 import zaxpby_f32
    A2, B2 = s1_complex_embed(np.asarray(A, np.complex64), np.asarray(B, np.complex64))
    H2 = s1_sgemm(A2, B2, p)
    return zaxpby_f32(alpha, H2[:, 0::2], H2[:, 1::2], beta, C)
