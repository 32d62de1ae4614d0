"""Pins of the oracle's Scheme I complex product by 4M (Sec. IV-B): the real
embedding holds exactly the four real products, the result is the correctly
rounded exact complex product whenever no slice pair is dropped, and the
error falls with p like the real scheme's."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from oracle import metrics


def _exact_complex(A, B):
    M, K = A.shape
    N = B.shape[1]
    F = Fraction
    re = [[sum(F(float(A[i, k].real)) * F(float(B[k, j].real)) - F(float(A[i, k].imag)) * F(float(B[k, j].imag))
               for k in range(K)) for j in range(N)] for i in range(M)]
    im = [[sum(F(float(A[i, k].real)) * F(float(B[k, j].imag)) + F(float(A[i, k].imag)) * F(float(B[k, j].real))
               for k in range(K)) for j in range(N)] for i in range(M)]
    return re, im


def test_embedding_holds_the_four_real_products():
    A = synth.complex_phi_matrix(3, 5, 1.0, 1, 2)
    B = synth.complex_phi_matrix(5, 4, 1.0, 3, 4)
    A2, B2 = oracle.s1_complex_embed(A, B)
    assert A2.shape == (3, 10) and B2.shape == (10, 8)
    re, im = _exact_complex(A, B)
    F = Fraction
    for i in range(3):
        for jj in range(8):
            v = sum(F(float(A2[i, k])) * F(float(B2[k, jj])) for k in range(10))
            assert v == (re if jj % 2 == 0 else im)[i][jj // 2]


@pytest.mark.parametrize("bits,p", [(6, 1), (14, 2), (22, 3)])
def test_exact_when_no_pair_is_dropped(bits, p):
    """Integer parts of at most 8 t - 2 bits fill t balanced digits; with
    2 t - 1 <= p every pair is kept and each part of the result is the
    correctly rounded exact value."""
    rng = np.random.default_rng(bits)
    M, N, K = 4, 3, 9
    lim = 2 ** bits
    A = rng.integers(-lim + 1, lim, (M, K)) + 1j * rng.integers(-lim + 1, lim, (M, K))
    B = rng.integers(-lim + 1, lim, (K, N)) + 1j * rng.integers(-lim + 1, lim, (K, N))
    A[:, 0] = lim - 1
    B[0, :] = lim - 1
    t = (bits + 2 + 7) // 8
    pp = max(p, 2 * t - 1)
    got = oracle.s1_zgemm(A, B, pp)
    re, im = _exact_complex(A, B)
    for i in range(M):
        for j in range(N):
            assert got[i, j].real == float(re[i][j]) and got[i, j].imag == float(im[i][j])


def test_error_falls_with_p_and_meets_fp64_at_p8():
    A = synth.complex_phi_matrix(6, 300, 1.0, 11, 12)
    B = synth.complex_phi_matrix(300, 5, 1.0, 13, 14)
    hi, lo = oracle.zgemm_dd(A, B)
    errs = [metrics.e_cw(oracle.s1_zgemm(A, B, p), hi, lo, A, B) for p in range(2, 9)]
    for a, b in zip(errs, errs[1:]):
        assert b < a / 64 or b < 1e-16, errs
    assert errs[-1] < 1e-15


def test_alpha_beta_zero_rows_and_nonfinite():
    A = synth.complex_phi_matrix(5, 7, 1.0, 21, 22)
    B = synth.complex_phi_matrix(7, 4, 1.0, 23, 24)
    C0 = synth.complex_phi_matrix(5, 4, 1.0, 25, 26)
    A[1] = 0
    B[3, 2] = complex(np.nan, 0.0)
    out = oracle.s1_zgemm(A, B, 6, alpha=0.5 - 2j, beta=1 + 1j, C=C0)
    base = oracle.s1_zgemm(A, B, 6)
    assert np.array_equal(out[1], oracle.scheme2.zaxpby(0.5 - 2j, base[1:2], 1 + 1j, C0[1:2])[0], equal_nan=True)
    assert np.isnan(base[:, 2].real).all() and np.isnan(base[:, 2].imag).all()
    assert not np.isnan(base[:, [0, 1, 3]]).any()
    assert (base[1, [0, 1, 3]] == 0).all()


def test_cgemm_small_integers_exact_and_binary32_rounding():
    rng = np.random.default_rng(5)
    A = (rng.integers(-60, 61, (4, 6)) + 1j * rng.integers(-60, 61, (4, 6))).astype(np.complex64)
    B = (rng.integers(-60, 61, (6, 3)) + 1j * rng.integers(-60, 61, (6, 3))).astype(np.complex64)
    got = oracle.s1_cgemm(A, B, 2)
    assert got.dtype == np.complex64
    assert np.array_equal(got, (A.astype(np.complex128) @ B.astype(np.complex128)).astype(np.complex64))
    # generic operands: each part is binary32 rounding of the exact embedded product when every pair is kept
    X = synth.complex_phi_matrix(3, 8, 1.0, 31, 32).astype(np.complex64)
    Y = synth.complex_phi_matrix(8, 2, 1.0, 33, 34).astype(np.complex64)
    re, im = _exact_complex(X, Y)
    got = oracle.s1_cgemm(X, Y, 8)
    for i in range(3):
        for j in range(2):
            assert abs(float(got[i, j].real) - float(re[i][j])) <= abs(float(re[i][j])) * 2.0 ** -23 + 1e-30
            assert abs(float(got[i, j].imag) - float(im[i][j])) <= abs(float(im[i][j])) * 2.0 ** -23 + 1e-30
