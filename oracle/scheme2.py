"""Ozaki Scheme II (CRT over INT8 residues) and its 3M complex form.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Steps, in the paper's order (Sec. II-C.2, Eqs. 4-8; complex: Sec. IV-B, Eq. 16):

1. moduli: the first s of the greedy descending pairwise-coprime list that
   starts at 256 (the paper names 256, 255, 253, ...);
2. power-of-two row scales 2^sigma_i for A and column scales 2^tau_j for B,
   chosen so that the CRT exactness condition 2 sum_h |a'||b'| < P holds;
3. integerise: A' = trunc(diag(2^sigma) A), B' = trunc(B diag(2^tau));
4. residues A'_l = A' mod m_l (symmetric representative, fits int8);
5. one integer product per modulus, reduced mod m_l (Eqs. 6-7);
6. CRT recombination (Eq. 8) with the symmetric lift mod P;
7. inverse scaling, rounded once to nearest-even, then alpha/beta.

Readings where the paper is silent (each also listed in the design notes):
* scale rule (paper: "power-of-two vectors" only): the row exponent bound
  nb_i with ||a_i||_2 < 2^nb_i is computed from the entries' exponents in
  integer arithmetic, and sigma_i = T_A - nb_i with T_A + T_B = ceil(log2 P) - 2;
  by Cauchy-Schwarz 2 sum|a'||b'| < 2^(T_A+T_B+1) <= P.
* residue range: symmetric, smod(x, m) in [-floor(m/2), ceil(m/2)-1], because
  [0, m-1] does not fit signed INT8 for m > 128;
* CRT sign: the symmetric lift smod(., P) (products may be negative);
* 3M: one shared per-row scale for the real and imaginary parts (so that the
  sum plane means A_re + A_im), bounded through |re| + |im|; the 3M
  combination is formed on the INT32 values and reduced mod m.
"""
from __future__ import annotations

import math
from fractions import Fraction
from typing import List, Tuple

import numpy as np

ZERO_EXP = -100000
NONFINITE_EXP = 100000


# ------------------------------------------------------------------ moduli

def moduli(s: int) -> List[int]:
    """First s moduli of the greedy descending pairwise-coprime list from 256."""
    if not 1 <= s <= 20:
        raise ValueError("s must be in [1, 20]")
    out: List[int] = []
    m = 256
    while len(out) < s:
        if all(math.gcd(m, q) == 1 for q in out):
            out.append(m)
        m -= 1
    return out


def crt_constants(s: int) -> Tuple[int, List[int], List[int]]:
    """P = prod m_l, and W_l = (P/m_l) q_l with q_l = (P/m_l)^-1 mod m_l (Eq. 8)."""
    return crt_constants_for(moduli(s))


def crt_constants_for(ms: List[int]) -> Tuple[int, List[int], List[int]]:
    """The same constants for any pairwise-coprime moduli list."""
    P = 1
    for m in ms:
        P *= m
    W = []
    for m in ms:
        Pm = P // m
        q = pow(Pm % m, -1, m) if m > 1 else 0
        W.append(Pm * q)
    return P, ms, W


def targets(s: int) -> Tuple[int, int]:
    """Bit budgets T_A, T_B with T_A + T_B = ceil(log2 P) - 2, T_A = floor(./2)."""
    P, _, _ = crt_constants(s)
    L = (P - 1).bit_length() - 2  # ceil(log2 P) - 2
    ta = L // 2
    return ta, L - ta


# ------------------------------------------------------------------ scales

def _expo(x: np.ndarray) -> np.ndarray:
    """frexp exponent (2^(e-1) <= |x| < 2^e) of each entry; 0 where x == 0."""
    _, e = np.frexp(x)
    return e.astype(np.int64)


def _norm_bound_exponents(ex: np.ndarray, present: np.ndarray, axis: int):
    """Given per-entry exponents ex (with |entry| < 2^ex) and a mask of the
    entries that take part, return (emax, nb) along `axis`:
      emax = max ex,  S = sum ceil(2^40 4^(ex - emax)),
      nb = emax + ceil((ceil(log2 S) - 40) / 2),
    so that the 2-norm of the line is below 2^nb.  Lines with no entry get
    emax = ZERO_EXP."""
    big = np.where(present, ex, np.iinfo(np.int64).min)
    emax = big.max(axis=axis, keepdims=True)
    d = np.where(present, ex - emax, 0)
    term = np.where(d >= -20, np.left_shift(np.int64(1), np.clip(40 + 2 * d, 0, 62)), 1)
    term = np.where(present, term, 0)
    S = term.sum(axis=axis)
    emax = emax.squeeze(axis)
    nb = np.zeros_like(S)
    for idx in np.ndindex(S.shape):
        s_ = int(S[idx])
        if s_ == 0:
            continue
        c = (s_ - 1).bit_length() - 40  # ceil(log2 S) - 40
        nb[idx] = int(emax[idx]) + (-((-c) // 2))  # + ceil(c / 2)
    emax = np.where(S == 0, ZERO_EXP, emax)
    return emax, nb


def _scales(axis: int, T: int, ex: np.ndarray, present: np.ndarray, finite: np.ndarray):
    emax, nb = _norm_bound_exponents(ex, present, axis)
    sig = np.where(emax == ZERO_EXP, 0, T - nb).astype(np.int64)
    bad = ~finite.all(axis=axis)
    return sig, bad


def row_scales(A: np.ndarray, T: int):
    """sigma_i (and a mask of rows holding a non-finite value) for real A."""
    A = np.asarray(A, np.float64)
    fin = np.isfinite(A)
    A0 = np.where(fin, A, 0.0)
    return _scales(1, T, _expo(A0), A0 != 0, fin)


def col_scales(B: np.ndarray, T: int):
    """tau_j (and a mask of non-finite columns) for real B."""
    B = np.asarray(B, np.float64)
    fin = np.isfinite(B)
    B0 = np.where(fin, B, 0.0)
    return _scales(0, T, _expo(B0), B0 != 0, fin)


def _complex_expo(X: np.ndarray):
    re, im = X.real, X.imag
    fin = np.isfinite(re) & np.isfinite(im)
    re = np.where(fin, re, 0.0)
    im = np.where(fin, im, 0.0)
    er = np.where(re != 0, _expo(re), np.iinfo(np.int32).min)
    ei = np.where(im != 0, _expo(im), np.iinfo(np.int32).min)
    present = (re != 0) | (im != 0)
    ex = np.where(present, np.maximum(er, ei) + 1, 0)  # |re| + |im| < 2^ex
    return ex, present, fin


def row_scales_complex(A: np.ndarray, T: int):
    """Shared sigma_i for the real and imaginary parts of row i of A."""
    A = np.asarray(A, np.complex128)
    ex, present, fin = _complex_expo(A)
    return _scales(1, T, ex, present, fin)


def col_scales_complex(B: np.ndarray, T: int):
    B = np.asarray(B, np.complex128)
    ex, present, fin = _complex_expo(B)
    return _scales(0, T, ex, present, fin)


# -------------------------------------------------------------- integerise

def integerise(X: np.ndarray, sig: np.ndarray, axis: int) -> np.ndarray:
    """trunc(x 2^sig) as an exact integer-valued float64 array (|.| < 2^77)."""
    X = np.asarray(X, np.float64)
    X = np.where(np.isfinite(X), X, 0.0)
    s = sig.reshape((-1, 1)) if axis == 1 else sig.reshape((1, -1))
    return np.trunc(np.ldexp(X, s.astype(np.int32)))


def smod(x, m):
    """Symmetric residue x - m floor((2x + m) / (2m)), in [-floor(m/2), ceil(m/2)-1]."""
    return x - m * ((2 * x + m) // (2 * m))


def residues(Xint: np.ndarray, m: int) -> np.ndarray:
    """Symmetric residues of an integer-valued float64 array, as int8."""
    r = np.fmod(Xint, float(m)).astype(np.int64)  # fmod is exact
    return smod(r, m).astype(np.int8)


# ---------------------------------------------------------------- products

def modular_product(RA: np.ndarray, RB: np.ndarray, m: int) -> np.ndarray:
    """Eqs. 6-7: C'_l = smod(RA RB, m) with an exact int64 product."""
    acc = RA.astype(np.int64) @ RB.astype(np.int64)
    return smod(acc, m).astype(np.int8)


def crt(Cl: List[np.ndarray], s: int) -> np.ndarray:
    """Eq. 8 with the symmetric lift: Z = smod(sum_l W_l C'_l, P) (object ints)."""
    return crt_for(Cl, moduli(s))


def crt_for(Cl: List[np.ndarray], ms: List[int]) -> np.ndarray:
    """Eq. 8 for any pairwise-coprime moduli list ms."""
    P, _, W = crt_constants_for(ms)
    acc = np.zeros(Cl[0].shape, dtype=object)
    for w, c in zip(W, Cl):
        acc = acc + c.astype(np.int64).astype(object) * w
    z = acc % P
    return np.where(2 * z >= P, z - P, z)


def scaled_round(z: int, E: int) -> float:
    """RN-even of z 2^E via Python's correctly rounded integer division."""
    try:
        if E >= 0:
            return float(z << E)
        return z / (1 << (-E))
    except OverflowError:
        return math.copysign(math.inf, z)


def _round_all(Z: np.ndarray, sig: np.ndarray, tau: np.ndarray) -> np.ndarray:
    M, N = Z.shape
    out = np.empty((M, N), np.float64)
    for i in range(M):
        si = int(sig[i])
        for j in range(N):
            out[i, j] = scaled_round(int(Z[i, j]), -si - int(tau[j]))
    return out


def _fma(a, b, c):
    """Correctly rounded fused multiply-add through exact rationals; a NaN or
    infinite operand propagates as in IEEE 754 (the product and sum are then
    not finite and no rounding question arises)."""
    if not (math.isfinite(a) and math.isfinite(b) and math.isfinite(c)):
        return a * b + c
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def axpby(alpha: float, H: np.ndarray, beta: float, C) -> np.ndarray:
    """alpha*H if beta == 0 (C not read), else fma(alpha, H, beta*C)."""
    if beta == 0.0:
        return alpha * H
    C = np.asarray(C, np.float64)
    bc = beta * C
    out = np.empty_like(H)
    for idx in np.ndindex(H.shape):
        out[idx] = _fma(alpha, float(H[idx]), float(bc[idx]))
    return out


# ------------------------------------------------------------------ DGEMM

def s2_prepare(A, B, s: int):
    """Scales, integerised operands and the per-modulus residue planes."""
    ta, tb = targets(s)
    sig, bad_r = row_scales(A, ta)
    tau, bad_c = col_scales(B, tb)
    Ai = integerise(A, sig, 1)
    Bi = integerise(B, tau, 0)
    ms = moduli(s)
    RA = [residues(Ai, m) for m in ms]
    RB = [residues(Bi, m) for m in ms]
    return dict(sig=sig, tau=tau, bad_r=bad_r, bad_c=bad_c, Ai=Ai, Bi=Bi, RA=RA, RB=RB, ms=ms)


def s2_dgemm(A, B, s: int, alpha=1.0, beta=0.0, C=None, return_parts=False):
    """Whole Scheme II DGEMM following steps 1-7."""
    st = s2_prepare(A, B, s)
    Cl = [modular_product(ra, rb, m) for ra, rb, m in zip(st["RA"], st["RB"], st["ms"])]
    Z = crt(Cl, s)
    H = _round_all(Z, st["sig"], st["tau"])
    H[st["bad_r"], :] = np.nan
    H[:, st["bad_c"]] = np.nan
    out = axpby(alpha, H, beta, C)
    if return_parts:
        st.update(Cl=Cl, Z=Z, H=H)
        return out, st
    return out


def s2_exact_definition(A, B, s: int) -> np.ndarray:
    """The plain definition the CRT path reproduces:
    RN(diag(2^-sigma) (A' B') diag(2^-tau)) with an exact big-integer product."""
    ta, tb = targets(s)
    sig, _ = row_scales(A, ta)
    tau, _ = col_scales(B, tb)
    Ai = integerise(A, sig, 1).astype(object)
    Bi = integerise(B, tau, 0).astype(object)
    Ai = np.vectorize(int, otypes=[object])(Ai)
    Bi = np.vectorize(int, otypes=[object])(Bi)
    Z = Ai @ Bi
    return _round_all(Z, sig, tau)


# ------------------------------------------------------------- 3M ZGEMM

def z3m_prepare(A, B, s: int):
    ta, tb = targets(s)
    A = np.asarray(A, np.complex128)
    B = np.asarray(B, np.complex128)
    sig, bad_r = row_scales_complex(A, ta)
    tau, bad_c = col_scales_complex(B, tb)
    Are, Aim = integerise(A.real, sig, 1), integerise(A.imag, sig, 1)
    Bre, Bim = integerise(B.real, tau, 0), integerise(B.imag, tau, 0)
    ms = moduli(s)
    planes = []
    for m in ms:
        r_re, r_im = residues(Are, m), residues(Aim, m)
        s_re, s_im = residues(Bre, m), residues(Bim, m)
        r_sum = smod(r_re.astype(np.int64) + r_im, m).astype(np.int8)
        s_sum = smod(s_re.astype(np.int64) + s_im, m).astype(np.int8)
        planes.append(((r_re, r_im, r_sum), (s_re, s_im, s_sum)))
    return dict(sig=sig, tau=tau, bad_r=bad_r, bad_c=bad_c, Are=Are, Aim=Aim,
                Bre=Bre, Bim=Bim, planes=planes, ms=ms)


def z3m_modular(RA, RB, m: int):
    """Eq. 16 per modulus: T1, T2, T3 reduced mod m, then
    C'_re = smod(T1 - T2), C'_im = smod(T3 - T1 - T2)."""
    (r_re, r_im, r_sum), (s_re, s_im, s_sum) = RA, RB
    T1 = smod(r_re.astype(np.int64) @ s_re.astype(np.int64), m)
    T2 = smod(r_im.astype(np.int64) @ s_im.astype(np.int64), m)
    T3 = smod(r_sum.astype(np.int64) @ s_sum.astype(np.int64), m)
    return smod(T1 - T2, m).astype(np.int8), smod(T3 - T1 - T2, m).astype(np.int8)


def zaxpby(alpha: complex, H: np.ndarray, beta: complex, C) -> np.ndarray:
    """Fixed fma sequence for complex alpha/beta:
      beta == 0: bc = 0 and C is not read; otherwise
        bc_re = fma(b_re, c_re, -(b_im c_im)),  bc_im = fma(b_re, c_im, b_im c_re);
      out_re = fma(a_re, h_re, fma(-a_im, h_im, bc_re)),
      out_im = fma(a_re, h_im, fma(a_im, h_re, bc_im))."""
    alpha = complex(alpha)
    beta = complex(beta)
    out = np.empty(H.shape, np.complex128)
    Cc = None if beta == 0 else np.asarray(C, np.complex128)
    for idx in np.ndindex(H.shape):
        h = H[idx]
        if beta == 0:
            bre = bim = 0.0
        else:
            c = Cc[idx]
            bre = _fma(beta.real, c.real, -(beta.imag * c.imag))
            bim = _fma(beta.real, c.imag, beta.imag * c.real)
        ore = _fma(alpha.real, h.real, _fma(-alpha.imag, h.imag, bre))
        oim = _fma(alpha.real, h.imag, _fma(alpha.imag, h.real, bim))
        out[idx] = complex(ore, oim)
    return out


def z3m_gemm(A, B, s: int, alpha=1.0, beta=0.0, C=None, return_parts=False):
    """Whole Scheme II 3M ZGEMM."""
    st = z3m_prepare(A, B, s)
    cre, cim = [], []
    for (RA, RB), m in zip(st["planes"], st["ms"]):
        r, i = z3m_modular(RA, RB, m)
        cre.append(r)
        cim.append(i)
    Zre, Zim = crt(cre, s), crt(cim, s)
    Hre = _round_all(Zre, st["sig"], st["tau"])
    Him = _round_all(Zim, st["sig"], st["tau"])
    H = Hre + 1j * Him
    H[st["bad_r"], :] = complex(np.nan, np.nan)
    H[:, st["bad_c"]] = complex(np.nan, np.nan)
    out = zaxpby(alpha, H, beta, C)
    if return_parts:
        st.update(Cre=cre, Cim=cim, Zre=Zre, Zim=Zim, H=H)
        return out, st
    return out


def z3m_exact_definition(A, B, s: int) -> np.ndarray:
    """Plain 4M definition: C'_re = A'_re B'_re - A'_im B'_im,
    C'_im = A'_re B'_im + A'_im B'_re (exact big integers), then RN(2^-sigma-tau .)."""
    st = z3m_prepare(A, B, s)
    big = np.vectorize(int, otypes=[object])
    ar, ai, br, bi = (big(st[k].astype(object)) for k in ("Are", "Aim", "Bre", "Bim"))
    Zre = ar @ br - ai @ bi
    Zim = ar @ bi + ai @ br
    return _round_all(Zre, st["sig"], st["tau"]) + 1j * _round_all(Zim, st["sig"], st["tau"])


# ------------------------------------------------------ sampled outputs only

def s2_entries(A, B, s: int, rows, cols, alpha=1.0, beta=0.0, cin=None) -> np.ndarray:
    """Scheme II outputs (rows[n], cols[n]) computed one by one with the same
    steps: full-row/column scales, integerise the needed row and column,
    residues, one modular dot product per modulus, CRT, one rounding."""
    A = np.asarray(A, np.float64)
    B = np.asarray(B, np.float64)
    ta, tb = targets(s)
    sig, bad_r = row_scales(A, ta)
    tau, bad_c = col_scales(B, tb)
    ms = moduli(s)
    out = np.empty(len(rows), np.float64)
    for n, (i, j) in enumerate(zip(rows, cols)):
        i, j = int(i), int(j)
        if bad_r[i] or bad_c[j]:
            h = math.nan
        else:
            a = integerise(A[i:i + 1], sig[i:i + 1], 1)
            b = integerise(B[:, j:j + 1], tau[j:j + 1], 0)
            Cl = [modular_product(residues(a, m), residues(b, m), m) for m in ms]
            z = int(crt(Cl, s)[0, 0])
            h = scaled_round(z, -int(sig[i]) - int(tau[j]))
        if beta == 0.0:
            out[n] = alpha * h
        else:
            out[n] = _fma(alpha, h, beta * float(cin[n]))
    return out


def z3m_entries(A, B, s: int, rows, cols) -> np.ndarray:
    """3M ZGEMM outputs (rows[n], cols[n]) one by one (alpha = 1, beta = 0)."""
    A = np.asarray(A, np.complex128)
    B = np.asarray(B, np.complex128)
    ta, tb = targets(s)
    sig, bad_r = row_scales_complex(A, ta)
    tau, bad_c = col_scales_complex(B, tb)
    ms = moduli(s)
    out = np.empty(len(rows), np.complex128)
    for n, (i, j) in enumerate(zip(rows, cols)):
        i, j = int(i), int(j)
        if bad_r[i] or bad_c[j]:
            out[n] = complex(math.nan, math.nan)
            continue
        ar = integerise(A[i:i + 1].real, sig[i:i + 1], 1)
        ai = integerise(A[i:i + 1].imag, sig[i:i + 1], 1)
        br = integerise(B[:, j:j + 1].real, tau[j:j + 1], 0)
        bi = integerise(B[:, j:j + 1].imag, tau[j:j + 1], 0)
        cre, cim = [], []
        for m in ms:
            r_re, r_im = residues(ar, m), residues(ai, m)
            s_re, s_im = residues(br, m), residues(bi, m)
            r_sum = smod(r_re.astype(np.int64) + r_im, m).astype(np.int8)
            s_sum = smod(s_re.astype(np.int64) + s_im, m).astype(np.int8)
            x, y = z3m_modular((r_re, r_im, r_sum), (s_re, s_im, s_sum), m)
            cre.append(x)
            cim.append(y)
        E = -int(sig[i]) - int(tau[j])
        h = complex(scaled_round(int(crt(cre, s)[0, 0]), E), scaled_round(int(crt(cim, s)[0, 0]), E))
        out[n] = zaxpby(1.0, np.array([h]), 0.0, None)[0]
    return out


# ------------------------------------------- binary32 operands and results

def rn_f32(x: Fraction) -> np.float32:
    """Round-to-nearest-even of an exact rational to binary32: 24 significant
    bits, gradual underflow at 2^-149, overflow to infinity."""
    if x == 0:
        return np.float32(0.0)
    neg = x < 0
    num, den = abs(x.numerator), x.denominator
    e = num.bit_length() - den.bit_length()  # 2^e <= |x| < 2^(e+1) after the correction
    if (num << max(0, -e)) < (den << max(0, e)):
        e -= 1
    sh = 23 - max(e, -126)  # q = |x| 2^sh has 24 bits (fewer when subnormal)
    n2, d2 = (num << sh, den) if sh >= 0 else (num, den << -sh)
    q, r = divmod(n2, d2)
    if 2 * r > d2 or (2 * r == d2 and q & 1):
        q += 1
    if q.bit_length() - sh > 128:
        v = math.inf
    else:
        v = math.ldexp(q, -sh)  # q <= 2^24: exact in binary64 and in binary32
    return np.float32(-v if neg else v)


def scaled_round_f32(z: int, E: int) -> np.float32:
    """RN-even of z 2^E to binary32."""
    return rn_f32(Fraction(z) * (Fraction(2) ** E))


def _fmaf(a, b, c) -> np.float32:
    """Correctly rounded binary32 fused multiply-add through exact rationals."""
    a, b, c = np.float32(a), np.float32(b), np.float32(c)
    if not (np.isfinite(a) and np.isfinite(b) and np.isfinite(c)):
        return np.float32(a * b + c)
    return rn_f32(Fraction(float(a)) * Fraction(float(b)) + Fraction(float(c)))


def _round_all_f32(Z: np.ndarray, sig: np.ndarray, tau: np.ndarray) -> np.ndarray:
    M, N = Z.shape
    out = np.empty((M, N), np.float32)
    for i in range(M):
        for j in range(N):
            out[i, j] = scaled_round_f32(int(Z[i, j]), -int(sig[i]) - int(tau[j]))
    return out


def axpby_f32(alpha: float, H: np.ndarray, beta: float, C) -> np.ndarray:
    """alpha*H if beta == 0 (C not read), else fmaf(alpha, H, beta*C), in binary32."""
    alpha, beta = np.float32(alpha), np.float32(beta)
    if beta == 0:
        return alpha * H
    bc = beta * np.asarray(C, np.float32)
    out = np.empty_like(H)
    for idx in np.ndindex(H.shape):
        out[idx] = _fmaf(alpha, H[idx], bc[idx])
    return out


def s2_sgemm(A, B, s: int, alpha=1.0, beta=0.0, C=None):
    """Scheme II SGEMM: steps 1-6 on the exactly widened binary32 operands,
    one rounding of Z 2^E to binary32, then alpha/beta in binary32."""
    A = np.asarray(A, np.float32).astype(np.float64)
    B = np.asarray(B, np.float32).astype(np.float64)
    st = s2_prepare(A, B, s)
    Cl = [modular_product(ra, rb, m) for ra, rb, m in zip(st["RA"], st["RB"], st["ms"])]
    H = _round_all_f32(crt(Cl, s), st["sig"], st["tau"])
    H[st["bad_r"], :] = np.nan
    H[:, st["bad_c"]] = np.nan
    return axpby_f32(alpha, H, beta, C)


def z3m_cgemm(A, B, s: int, alpha=1.0, beta=0.0, C=None):
    """Scheme II 3M CGEMM: the 3M steps on the exactly widened complex64
    operands, binary32 roundings, and the fixed FMA sequence of zaxpby in
    binary32 (fmaf)."""
    A = np.asarray(A, np.complex64).astype(np.complex128)
    B = np.asarray(B, np.complex64).astype(np.complex128)
    st = z3m_prepare(A, B, s)
    cre, cim = [], []
    for (RA, RB), m in zip(st["planes"], st["ms"]):
        r, i = z3m_modular(RA, RB, m)
        cre.append(r)
        cim.append(i)
    Hre = _round_all_f32(crt(cre, s), st["sig"], st["tau"])
    Him = _round_all_f32(crt(cim, s), st["sig"], st["tau"])
    Hre[st["bad_r"], :] = np.nan
    Him[st["bad_r"], :] = np.nan
    Hre[:, st["bad_c"]] = np.nan
    Him[:, st["bad_c"]] = np.nan
    return zaxpby_f32(alpha, Hre, Him, beta, C)


def zaxpby_f32(alpha: complex, Hre: np.ndarray, Him: np.ndarray, beta: complex, C) -> np.ndarray:
    """The fixed FMA sequence of zaxpby in binary32 (fmaf), for the binary32
    parts Hre, Him of the complex result; beta == 0: C is not read."""
    al, be = complex(alpha), complex(beta)
    ar, ai, br, bi = (np.float32(v) for v in (al.real, al.imag, be.real, be.imag))
    out = np.empty(Hre.shape, np.complex64)
    Cc = None if be == 0 else np.asarray(C, np.complex64)
    for idx in np.ndindex(Hre.shape):
        hr, hi = np.float32(Hre[idx]), np.float32(Him[idx])
        if be == 0:
            bre = bim = np.float32(0.0)
        else:
            c = Cc[idx]
            cr, ci = np.float32(c.real), np.float32(c.imag)
            bre = _fmaf(br, cr, -(bi * ci))
            bim = _fmaf(br, ci, bi * cr)
        ore = _fmaf(ar, hr, _fmaf(-ai, hi, bre))
        oim = _fmaf(ar, hi, _fmaf(ai, hr, bim))
        out[idx] = np.complex64(complex(float(ore), float(oim)))
    return out
