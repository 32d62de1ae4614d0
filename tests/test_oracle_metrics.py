"""Pins of the oracle's error metrics, of its exact shift-reduce integer Z
(Eq. 3 before the rounding) and of the fixed complex FMA sequence that the
complex alpha/beta update follows.

Each expected value is either a worked example whose result is written out
by hand below, a closed form, or a property of exact arithmetic checked with
Python fractions / big integers, chosen so that a plausible slip (swapped
real/imaginary scales, a dropped term, an FMA taken in the other order, a
wrong shift) changes the result."""
import ctypes
import ctypes.util
import math
import random
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from oracle import metrics
from oracle import scheme2 as s2

_libm = ctypes.CDLL(ctypes.util.find_library("m"))
_libm.fma.restype = ctypes.c_double
_libm.fma.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double]


def libm_fma(a, b, c):
    """The C library's correctly rounded fused multiply-add (glibc fma)."""
    return _libm.fma(a, b, c)


# ------------------------------------------------------------- E_cw, complex

def test_complex_e_cw_worked_example():
    """A = [1+2i, 3-i], B = [1-i; 2+0.5i]:
    real part  sum(Ar Br - Ai Bi) = 3 + 6.5 = 9.5, scale sum(|Ar||Br| + |Ai||Bi|) = 3 + 6.5 = 9.5;
    imag part  sum(Ar Bi + Ai Br) = 1 - 0.5 = 0.5, scale sum(|Ar||Bi| + |Ai||Br|) = 3 + 3.5 = 6.5.
    With errors 3 2^-49 (real) and 78 2^-53 (imag) the ratios are
    3 2^-49 / 9.5 ~ 1.263 2^-50 and 78 2^-53 / 6.5 = 12 2^-53 = 1.5 2^-50,
    so E_cw = 1.5 2^-50.  Swapping the two scales would give 3 2^-49 / 6.5
    ~ 1.846 2^-50; scaling by complex moduli gives yet another value."""
    A = np.array([[1 + 2j, 3 - 1j]])
    B = np.array([[1 - 1j], [2 + 0.5j]])
    hi = np.array([[9.5 + 0.5j]])
    lo = np.zeros_like(hi)
    C = np.array([[complex(9.5 + 3 * 2.0 ** -49, 0.5 - 78 * 2.0 ** -53)]])
    assert C[0, 0].real - 9.5 == 3 * 2.0 ** -49 and 0.5 - C[0, 0].imag == 78 * 2.0 ** -53
    assert metrics.e_cw(C, hi, lo, A, B) == 1.5 * 2.0 ** -50
    # the low part of the reference is subtracted too
    lo2 = np.array([[complex(2.0 ** -49, 0.0)]])
    assert metrics.e_cw(C, hi, lo2, A, B) == max(2 * 2.0 ** -49 / 9.5, 1.5 * 2.0 ** -50)


def test_complex_e_cw_against_exact_fractions():
    """Random complex data: the metric equals the definition evaluated in
    exact rationals (the reference being the exact product) to within the
    few roundings of the floating-point evaluation."""
    A = synth.complex_phi_matrix(4, 7, 1.5, 11, 12)
    B = synth.complex_phi_matrix(7, 5, 1.5, 13, 14)
    rng = np.random.default_rng(5)
    hi, lo = oracle.zgemm_dd(A, B)
    pert = (rng.integers(-40, 40, size=hi.shape) + 1j * rng.integers(-40, 40, size=hi.shape)) * 2.0 ** -50
    C = hi * (1 + pert)
    F = Fraction
    worst = F(0)
    for i in range(4):
        for j in range(5):
            re = sum(F(A[i, k].real) * F(B[k, j].real) - F(A[i, k].imag) * F(B[k, j].imag) for k in range(7))
            im = sum(F(A[i, k].real) * F(B[k, j].imag) + F(A[i, k].imag) * F(B[k, j].real) for k in range(7))
            sr = sum(abs(F(A[i, k].real)) * abs(F(B[k, j].real)) + abs(F(A[i, k].imag)) * abs(F(B[k, j].imag))
                     for k in range(7))
            si = sum(abs(F(A[i, k].real)) * abs(F(B[k, j].imag)) + abs(F(A[i, k].imag)) * abs(F(B[k, j].real))
                     for k in range(7))
            worst = max(worst, abs(F(C[i, j].real) - re) / sr, abs(F(C[i, j].imag) - im) / si)
    got = metrics.e_cw(C, hi, lo, A, B)
    assert abs(F(got) - worst) <= worst * F(1, 2 ** 40), (got, float(worst))


def test_complex_e_cw_skips_zero_scale_and_nonfinite():
    A = np.array([[1 + 0j, 0j], [0j, 0j]])
    B = np.array([[2 + 0j], [5 + 0j]])
    hi = np.array([[2 + 0j], [0j]])
    lo = np.zeros_like(hi)
    # imag scale of row 0 is 0 (no imaginary parts): its error is left out; row 1 has no scale at all
    C = np.array([[complex(2 + 2.0 ** -51, 1.0)], [complex(np.nan, np.nan)]])
    assert metrics.e_cw(C, hi, lo, A, B) == 2.0 ** -52


# --------------------------------------------------------------- E_nw, bits

def test_e_nw_closed_forms():
    # C = ref (1 + d) elementwise: E_nw = |d|
    ref = np.array([[3.0, 0.0], [0.0, -4.0]])
    d = 2.0 ** -20
    assert metrics.e_nw(ref * (1 + d), ref, np.zeros_like(ref)) == d
    # complex: |3 + 4i| = 5, the error (3 + 4i) 2^-30 has modulus 5 2^-30
    zr = np.array([[3 + 4j]])
    assert metrics.e_nw(zr * (1 + 2.0 ** -30), zr, np.zeros_like(zr)) == 2.0 ** -30
    # one error of 2^-30 against ||ref||_F = sqrt(2)
    eye = np.eye(2)
    got = metrics.e_nw(eye + np.array([[2.0 ** -30, 0], [0, 0]]), eye, np.zeros_like(eye))
    assert abs(got - 2.0 ** -30 / math.sqrt(2)) <= 2.0 ** -30 * 2.0 ** -52
    # the low part counts: C = hi exactly, lo = 2^-60 on one entry of ref = [[1]]
    assert metrics.e_nw(np.array([[1.0]]), np.array([[1.0]]), np.array([[2.0 ** -60]])) == 2.0 ** -60


def test_e_nw_against_exact_fractions():
    rng = np.random.default_rng(9)
    ref = rng.standard_normal((6, 5))
    C = ref + rng.integers(-1000, 1000, size=ref.shape) * 2.0 ** -60
    num = sum((Fraction(float(C[i, j])) - Fraction(float(ref[i, j]))) ** 2 for i in range(6) for j in range(5))
    den = sum(Fraction(float(ref[i, j])) ** 2 for i in range(6) for j in range(5))
    expect = math.sqrt(float(num / den))
    got = metrics.e_nw(C, ref, np.zeros_like(ref))
    assert abs(got - expect) <= expect * 2.0 ** -48


def test_bits_and_median():
    assert metrics.bits(2.0 ** -40) == 40.0
    assert metrics.bits(0.0) == math.inf
    assert abs(metrics.bits(0.75 * 2.0 ** -10) - (10 + math.log2(4 / 3))) < 1e-12
    ref = np.array([1.0, 2.0, 4.0, 0.0, 8.0])
    C = ref + np.array([2.0 ** -40, 2.0 ** -37, 2.0 ** -44, 1.0, 8 * 2.0 ** -38])
    # relative errors 2^-40, 2^-38, 2^-46, (zero reference skipped), 2^-38: the median of
    # the four is the mean of the middle two, (2^-40 + 2^-38) / 2
    assert metrics.median_rel(C, ref, np.zeros_like(ref)) == (2.0 ** -40 + 2.0 ** -38) / 2


# ----------------------------------------------------- Scheme I integer Z

def test_s1_z_equals_exact_product_when_no_pair_is_dropped():
    """With integer entries of at most 7 bits only the two leading slices are
    nonzero, so at p = 4 no slice pair is dropped and Z 2^E (E = e_i + f_j -
    12 - 8(p-1)) is the exact product: checked against big-integer dot
    products.  A wrong shift or a dropped diagonal changes Z."""
    p = 4
    rng = np.random.default_rng(21)
    M, N, K = 5, 4, 19
    A = rng.integers(-127, 128, size=(M, K)).astype(np.float64) * 2.0 ** rng.integers(-3, 4, size=(M, 1))
    B = rng.integers(-127, 128, size=(K, N)).astype(np.float64) * 2.0 ** rng.integers(-3, 4, size=(1, N))
    e = oracle.s1_row_exponents(A)
    f = oracle.s1_col_exponents(B)
    D = oracle.s1_digits_a(A, e, p)
    E = oracle.s1_digits_b(B, f, p)
    assert not D[2:].any() and not E[2:].any()
    Z = oracle.s1_z(oracle.s1_diagonals(D, E))
    for i in range(M):
        for j in range(N):
            exact = sum(Fraction(float(A[i, k])) * Fraction(float(B[k, j])) for k in range(K))
            sc = oracle.s1_scale_exponent(int(e[i]), int(f[j]), p)
            assert Fraction(Z[i * N + j]) * Fraction(2) ** sc == exact


def test_s1_z_full_range_and_reconstruct_consistency():
    """Z over diagonals near the int64 limits, against big integers, and the
    reconstruction is the one rounding of that Z (the correctly rounded
    division of Python integers)."""
    p = 8
    rnd = random.Random(4)
    Cd = np.empty((p, 3, 3), np.int64)
    for d in range(p):
        for i in range(3):
            for j in range(3):
                Cd[d, i, j] = rnd.choice([2 ** 62 - 1, -(2 ** 62), rnd.randint(-(2 ** 40), 2 ** 40), 0])
    Z = oracle.s1_z(Cd)
    for i in range(3):
        for j in range(3):
            ref = 0
            for d in range(p):
                ref = ref * 256 + int(Cd[d, i, j])
            assert Z[i * 3 + j] == ref
    e = np.array([0, 5, -7], np.int32)
    f = np.array([3, -2, 1], np.int32)
    H = oracle.s1_reconstruct(np.clip(Cd, -(2 ** 31), 2 ** 31 - 1), e, f)
    Zc = oracle.s1_z(np.clip(Cd, -(2 ** 31), 2 ** 31 - 1))
    for i in range(3):
        for j in range(3):
            E = oracle.s1_scale_exponent(int(e[i]), int(f[j]), p)
            z = Zc[i * 3 + j]
            want = float(z << E) if E >= 0 else z / (1 << -E)
            assert H[i, j] == want


# ------------------------------------------------- complex alpha/beta update

T = 1.0 + 2.0 ** -30  # T * T = 1 + 2^-29 + 2^-60, which rounds to 1 + 2^-29


def test_zaxpby_worked_examples():
    """Hand-evaluated cases in which each FMA of the documented sequence
    decides the result:
      alpha = T(1 + i), h = T(1 + i), beta = 0:
        out_re = fma(T, T, RN(-T T)) = (1 + 2^-29 + 2^-60) - (1 + 2^-29) = 2^-60
        (the other order, fma(-T, T, RN(T T)), gives -2^-60; without FMAs 0)
        out_im = fma(T, T, RN(T T)) = RN(2 + 2^-28 + 2^-60) = 2 + 2^-28;
      alpha = T(1 - i): out_re = 2 + 2^-28, out_im = fma(T, T, RN(-T T)) = 2^-60;
      alpha = 0, beta = T(1 + i), c = T(1 + i):
        bc_re = fma(T, T, -RN(T T)) = 2^-60, bc_im = fma(T, T, RN(T T)) = 2 + 2^-28."""
    h = np.array([[complex(T, T)]])
    out = s2.zaxpby(complex(T, T), h, 0.0, None)[0, 0]
    assert out.real == 2.0 ** -60 and out.imag == 2.0 + 2.0 ** -28
    out = s2.zaxpby(complex(T, -T), h, 0.0, None)[0, 0]
    assert out.real == 2.0 + 2.0 ** -28 and out.imag == 2.0 ** -60
    out = s2.zaxpby(0.0, h, complex(T, T), np.array([[complex(T, T)]]))[0, 0]
    assert out.real == 2.0 ** -60 and out.imag == 2.0 + 2.0 ** -28
    # beta == 0: C is not read
    assert np.array_equal(s2.zaxpby(1.0, h, 0.0, np.full((1, 1), complex(np.nan, np.nan))), h)


def test_zaxpby_matches_libm_fma_sequence():
    """Random operands: every output equals the documented sequence evaluated
    with the C library's fma, bit for bit."""
    rng = np.random.default_rng(17)
    H = rng.standard_normal((8, 8)) + 1j * rng.standard_normal((8, 8))
    C = rng.standard_normal((8, 8)) + 1j * rng.standard_normal((8, 8))
    for alpha, beta in [(1.3 - 0.7j, 0.25 + 2.5j), (-2.0 + 1e-9j, 1.0 + 0j), (0.1 + 0.2j, -3.0 - 1.1j)]:
        out = s2.zaxpby(alpha, H, beta, C)
        for idx in np.ndindex(H.shape):
            c, hh = C[idx], H[idx]
            bre = libm_fma(beta.real, c.real, -(beta.imag * c.imag))
            bim = libm_fma(beta.real, c.imag, beta.imag * c.real)
            ore = libm_fma(alpha.real, hh.real, libm_fma(-alpha.imag, hh.imag, bre))
            oim = libm_fma(alpha.real, hh.imag, libm_fma(alpha.imag, hh.real, bim))
            assert out[idx].real == ore and out[idx].imag == oim, (alpha, beta, idx)


def test_real_axpby_matches_libm_fma():
    rng = np.random.default_rng(18)
    H = rng.standard_normal((6, 7))
    C = rng.standard_normal((6, 7))
    out = s2.axpby(1.7, H, -0.3, C)
    for idx in np.ndindex(H.shape):
        assert out[idx] == libm_fma(1.7, H[idx], -0.3 * C[idx])
    assert np.array_equal(s2.axpby(2.0, H, 0.0, np.full_like(C, np.nan)), 2.0 * H)
