"""Pins of the reference products: naive FP64 and double-double against
exact rational arithmetic on small shapes."""
from fractions import Fraction

import numpy as np

import oracle
import synth


def _exact(A, B):
    M, K = A.shape
    N = B.shape[1]
    return [[sum(Fraction(float(A[i, k])) * Fraction(float(B[k, j])) for k in range(K))
             for j in range(N)] for i in range(M)]


def test_dd_matches_exact_product():
    A = synth.phi_matrix(6, 50, 3.0, 1)
    B = synth.phi_matrix(50, 7, 3.0, 2)
    hi, lo = oracle.gemm_dd(A, B)
    X = _exact(A, B)
    absAB = np.abs(A) @ np.abs(B)
    for i in range(6):
        for j in range(7):
            err = abs(Fraction(float(hi[i, j])) + Fraction(float(lo[i, j])) - X[i][j])
            assert err <= Fraction(float(absAB[i, j])) * Fraction(1, 2 ** 98)
            assert float(X[i][j]) == hi[i, j] or abs(float(X[i][j]) - hi[i, j]) <= abs(hi[i, j]) * 2 ** -52


def test_naive_within_rounding_bound():
    A = synth.phi_matrix(5, 40, 1.0, 3)
    B = synth.phi_matrix(40, 6, 1.0, 4)
    C = oracle.gemm_naive(A, B)
    X = _exact(A, B)
    absAB = np.abs(A) @ np.abs(B)
    K = 40
    gamma = K * 2.0 ** -53 / (1 - K * 2.0 ** -53)
    for i in range(5):
        for j in range(6):
            assert abs(Fraction(float(C[i, j])) - X[i][j]) <= Fraction(gamma * absAB[i, j] * (1 + 1e-12))


def test_zdd_matches_exact_product():
    A = synth.complex_phi_matrix(4, 20, 1.0, 5, 6)
    B = synth.complex_phi_matrix(20, 3, 1.0, 7, 8)
    hi, lo = oracle.zgemm_dd(A, B)
    for i in range(4):
        for j in range(3):
            re = sum(Fraction(float(A[i, k].real)) * Fraction(float(B[k, j].real))
                     - Fraction(float(A[i, k].imag)) * Fraction(float(B[k, j].imag)) for k in range(20))
            im = sum(Fraction(float(A[i, k].real)) * Fraction(float(B[k, j].imag))
                     + Fraction(float(A[i, k].imag)) * Fraction(float(B[k, j].real)) for k in range(20))
            scale = Fraction(float((np.abs(A[i]) @ np.abs(B[:, j])).real)) * 2
            assert abs(Fraction(float(hi[i, j].real)) + Fraction(float(lo[i, j].real)) - re) <= scale * Fraction(1, 2 ** 98)
            assert abs(Fraction(float(hi[i, j].imag)) + Fraction(float(lo[i, j].imag)) - im) <= scale * Fraction(1, 2 ** 98)


def test_error_metric_definition():
    A = np.array([[1.0, 2.0]])
    B = np.array([[3.0], [-1.0]])
    hi = np.array([[1.0]])
    lo = np.array([[0.0]])
    C = np.array([[1.0 + 5 * 2.0 ** -52]])
    # |C - ref| / (|A||B|) = 5 2^-52 / 5
    assert oracle.metrics.e_cw(C, hi, lo, A, B) == 2.0 ** -52
