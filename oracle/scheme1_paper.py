"""Scheme I with the slice format the paper adopts: a signed leading slice and
unsigned trailing slices (Sec. II-C.1, Eq. 1; Sec. VI).

TEST INFRASTRUCTURE ONLY (see the package docstring).  The library itself
slices differently (balanced signed digits of the rounded value); this
module exists so that the two formats can be compared on the same inputs.

Format, with beta = 8: each row of A is scaled by 2^-e_i (e_i the row
exponent, |a| < 2^e_i), so x = a 2^-e_i lies in (-1, 1).  The slices are the
floor digits of x 2^7:
    d_0 = floor(x 2^7)                     in [-128, 127]  (signed, SINT8)
    d_t = floor(r_(t-1) 2^8),  r_t = r_(t-1) 2^8 - d_t,  r_0 = x 2^7 - d_0,
                                           in [0, 255]     (unsigned, UINT8)
so x 2^7 = d_0 + sum_t d_t 2^-8t + (a residual below 2^-8(p-1)): 8p - 1
bits in all, each slice worth beta = 8 bits except the leading one, and the
digits do not depend on p (truncation keeps the prefix).  B is split the same
way along its columns.  Diagonals C_d = sum_{t+u=d} D_t E_u (Eq. 2) are exact
integers; the shift-reduce (Eq. 3) is done exactly, Z = sum_d 2^8(p-1-d) C_d,
and rounded once: C = RN(Z 2^(e_i + f_j - 14 - 8(p-1))).

On signed-only INT8 hardware an unsigned digit u is stored as v = u - 128 and
u w = v w + 128 v + 128 w + 128^2 (and d_0 u = d_0 v + 128 d_0), so every
pair product becomes a signed INT8 GEMM plus rank-1 corrections from row and
column sums; `diagonals_signed_storage` evaluates that form, which must give
the same integers.
"""
from __future__ import annotations

import numpy as np

from . import s1_col_exponents, s1_row_exponents
from .scheme2 import scaled_round

ZERO_EXP = -100000
NONFINITE_EXP = 100000


def _fixed(X: np.ndarray, e: np.ndarray, p: int, axis: int) -> np.ndarray:
    """floor(x 2^(8p-1)) with x = X 2^-e along `axis`, as Python integers
    (object array); lines with a sentinel exponent give 0."""
    X = np.asarray(X, np.float64)
    e = np.asarray(e, np.int64)
    live = (e != ZERO_EXP) & (e != NONFINITE_EXP)
    sh = np.where(live, 8 * p - 1 - e, 0)
    sh = sh.reshape((-1, 1)) if axis == 1 else sh.reshape((1, -1))
    live2 = live.reshape((-1, 1)) if axis == 1 else live.reshape((1, -1))
    X0 = np.where(np.isfinite(X) & live2, X, 0.0)
    # |x| < 1, so |x 2^(8p-1)| < 2^63: the scaling by a power of two and the
    # floor are exact in binary64 (the scaled value has at most 53 bits)
    Y = np.floor(np.ldexp(X0, sh.astype(np.int32)))
    return np.vectorize(int, otypes=[object])(Y)


def digits(X: np.ndarray, e: np.ndarray, p: int, axis: int) -> np.ndarray:
    """Slices [p][rows][cols] (int16: d_0 in [-128, 127], d_t in [0, 255])."""
    F = _fixed(X, e, p, axis)
    out = np.empty((p,) + F.shape, np.int16)
    for t in range(p):
        shift = 8 * (p - 1 - t)
        if t == 0:
            out[0] = np.vectorize(lambda z: z >> shift, otypes=[np.int64])(F)
        else:
            out[t] = np.vectorize(lambda z: (z >> shift) & 255, otypes=[np.int64])(F)
    return out


def diagonals(D: np.ndarray, E: np.ndarray) -> np.ndarray:
    """C_d = sum_{t <= d} D_t E_{d-t} (int64, exact: |terms| <= 255^2 K)."""
    p = D.shape[0]
    M, N = D.shape[1], E.shape[2]
    Cd = np.zeros((p, M, N), np.int64)
    for d in range(p):
        for t in range(d + 1):
            Cd[d] += D[t].astype(np.int64) @ E[d - t].astype(np.int64)
    return Cd


def diagonals_signed_storage(D: np.ndarray, E: np.ndarray) -> np.ndarray:
    """The same diagonals as a signed-only INT8 machine forms them: unsigned
    digits u stored as u - 128, each pair product a signed INT8 GEMM, plus
    the rank-1 corrections 128 rowsum + 128 colsum + 128^2 K."""
    p, M, K = D.shape
    N = E.shape[2]
    SD = D.astype(np.int64).copy()
    SE = E.astype(np.int64).copy()
    SD[1:] -= 128
    SE[1:] -= 128
    assert SD.min() >= -128 and SD.max() <= 127 and SE.min() >= -128 and SE.max() <= 127
    Cd = np.zeros((p, M, N), np.int64)
    for d in range(p):
        for t in range(d + 1):
            u = d - t
            acc = SD[t] @ SE[u]
            if u >= 1:  # stored B digit is w - 128: add 128 sum_k (A digit)
                acc += 128 * D[t].astype(np.int64).sum(axis=1, keepdims=True)
            if t >= 1:  # stored A digit is v - 128: add 128 sum_k (stored B digit)
                acc += 128 * SE[u].sum(axis=0, keepdims=True)
            Cd[d] += acc
    return Cd


def reconstruct(Cd: np.ndarray, e: np.ndarray, f: np.ndarray) -> np.ndarray:
    """Exact Z = sum_d 2^8(p-1-d) C_d, one rounding of Z 2^(e+f-14-8(p-1))."""
    p, M, N = Cd.shape
    out = np.empty((M, N), np.float64)
    for i in range(M):
        for j in range(N):
            ei, fj = int(e[i]), int(f[j])
            if ei in (ZERO_EXP, NONFINITE_EXP) or fj in (ZERO_EXP, NONFINITE_EXP):
                out[i, j] = np.nan if NONFINITE_EXP in (ei, fj) else 0.0
                continue
            z = 0
            for d in range(p):
                z = z * 256 + int(Cd[d, i, j])
            out[i, j] = scaled_round(z, ei + fj - 14 - 8 * (p - 1))
    return out


def dgemm(A: np.ndarray, B: np.ndarray, p: int) -> np.ndarray:
    """Whole Scheme I DGEMM in the paper's slice format (alpha 1, beta 0)."""
    e = s1_row_exponents(A)
    f = s1_col_exponents(B)
    D = digits(A, e, p, 1)
    E = digits(B, f, p, 0)
    return reconstruct(diagonals(D, E), e, f)


def digits_signed7(X: np.ndarray, e: np.ndarray, p: int, axis: int) -> np.ndarray:
    """The original signed-everywhere slices (beta = 7, Sec. II-C.1): the
    base-128 digits of trunc(|x| 2^7p) carrying the sign of x, each in
    [-127, 127], so x = sum_t d_t 2^-7(t+1) to within 2^-7p."""
    X = np.asarray(X, np.float64)
    e = np.asarray(e, np.int64)
    live = (e != ZERO_EXP) & (e != NONFINITE_EXP)
    sh = np.where(live, 7 * p - e, 0)
    sh = sh.reshape((-1, 1)) if axis == 1 else sh.reshape((1, -1))
    live2 = live.reshape((-1, 1)) if axis == 1 else live.reshape((1, -1))
    X0 = np.where(np.isfinite(X) & live2, X, 0.0)
    T = np.trunc(np.ldexp(X0, sh.astype(np.int32)))  # |x| 2^7p < 2^56: exact
    mag = np.vectorize(lambda z: abs(int(z)), otypes=[object])(T)
    sgn = np.sign(T).astype(np.int64)
    out = np.empty((p,) + X.shape, np.int16)
    for t in range(p):
        shift = 7 * (p - 1 - t)
        out[t] = sgn * np.vectorize(lambda z: (z >> shift) & 127, otypes=[np.int64])(mag)
    return out


def dgemm_signed7(A: np.ndarray, B: np.ndarray, p: int) -> np.ndarray:
    """Scheme I with the signed 7-bit slices: C_d as above, Z = sum_d
    2^7(p-1-d) C_d, one rounding of Z 2^(e_i + f_j - 7(p+1))."""
    e = s1_row_exponents(A)
    f = s1_col_exponents(B)
    Cd = diagonals(digits_signed7(A, e, p, 1), digits_signed7(B, f, p, 0))
    M, N = Cd.shape[1], Cd.shape[2]
    out = np.empty((M, N), np.float64)
    for i in range(M):
        for j in range(N):
            ei, fj = int(e[i]), int(f[j])
            if ei in (ZERO_EXP, NONFINITE_EXP) or fj in (ZERO_EXP, NONFINITE_EXP):
                out[i, j] = np.nan if NONFINITE_EXP in (ei, fj) else 0.0
                continue
            z = 0
            for d in range(p):
                z = z * 128 + int(Cd[d, i, j])
            out[i, j] = scaled_round(z, ei + fj - 7 * (p + 1))
    return out
