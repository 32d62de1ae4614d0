"""The paper's Scheme I slice format (signed leading slice, unsigned trailing
slices, beta = 8; Sec. II-C.1, Sec. VI) in the oracle, pinned by exact
arithmetic, and compared with the library's balanced digits and with the
original signed 7-bit slices on the headline workload's distribution.

The comparison is the evidence behind the library's choice of slice format:
on signed-only INT8 MFMA the balanced digits need no rank-1 corrections, and
their dropped slice pairs have random signs that cancel over K, while the
floor digits of the paper's format are all non-negative past the first
(large even for small negative entries), so their dropped pairs add up."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from oracle import metrics
from oracle import scheme1_paper as sp


def test_digits_worked_examples():
    """x = +-(1 - 2^-53) at p = 8: floor(x 2^63) = +-(2^63 - 2^10), whose
    bytes are 7F FF FF FF FF FF FC 00 and (two's complement) 80 00 00 00 00 00
    04 00; x = -1/2 gives d_0 = -64 and nothing else."""
    X = np.array([[1 - 2.0 ** -53, -(1 - 2.0 ** -53), -0.5]])
    e = np.array([0], np.int32)
    D = sp.digits(X, e, 8, 1)[:, 0, :]
    assert list(D[:, 0]) == [127, 255, 255, 255, 255, 255, 252, 0]
    assert list(D[:, 1]) == [-128, 0, 0, 0, 0, 0, 4, 0]
    assert list(D[:, 2]) == [-64, 0, 0, 0, 0, 0, 0, 0]


@pytest.mark.parametrize("p", [1, 3, 8])
def test_digits_sum_back_ranges_and_prefix(p):
    A = synth.phi_matrix(6, 40, 2.0, 77)
    A[2, 5] = 0.0
    e = oracle.s1_row_exponents(A)
    D = sp.digits(A, e, p, 1)
    assert D[0].min() >= -128 and D[0].max() <= 127
    if p > 1:
        assert D[1:].min() >= 0 and D[1:].max() <= 255
    for i in range(6):
        for k in range(40):
            x = Fraction(float(A[i, k])) / Fraction(2) ** int(e[i])
            val = sum(Fraction(int(D[t, i, k])) / Fraction(2) ** (7 + 8 * t) for t in range(p))
            scaled = x * 2 ** (8 * p - 1)
            floor = scaled.numerator // scaled.denominator
            assert val == Fraction(floor, 2 ** (8 * p - 1))  # x truncated (floor) to 8p - 1 bits
            assert 0 <= x - val < Fraction(1, 2 ** (8 * p - 1))
    if p < 8:
        assert np.array_equal(sp.digits(A, e, p + 1, 1)[:p], D)  # digits do not depend on p


def test_signed_storage_with_rank1_corrections_gives_the_same_diagonals():
    A = synth.phi_matrix(5, 70, 1.5, 78)
    B = synth.phi_matrix(70, 4, 1.5, 79)
    p = 8
    D = sp.digits(A, oracle.s1_row_exponents(A), p, 1)
    E = sp.digits(B, oracle.s1_col_exponents(B), p, 0)
    assert np.array_equal(sp.diagonals_signed_storage(D, E), sp.diagonals(D, E))


@pytest.mark.parametrize("bits,p", [(7, 1), (15, 3), (23, 5)])
def test_exact_when_no_pair_is_dropped(bits, p):
    """Integer entries of b bits (row maximum 2^b - 1) occupy the leading
    ceil((b - 7) / 8) + 1 digits; with p large enough for every pair the
    result is RN of the exact product."""
    rng = np.random.default_rng(bits)
    M, N, K = 4, 5, 30
    A = rng.integers(-(2 ** bits) + 1, 2 ** bits, size=(M, K)).astype(np.float64)
    B = rng.integers(-(2 ** bits) + 1, 2 ** bits, size=(K, N)).astype(np.float64)
    A[:, 0] = 2 ** bits - 1
    B[0, :] = 2 ** bits - 1
    got = sp.dgemm(A, B, p)
    for i in range(M):
        for j in range(N):
            exact = sum(Fraction(int(A[i, k])) * int(B[k, j]) for k in range(K))
            assert got[i, j] == float(exact)


def test_signed7_digits_sum_back():
    A = synth.phi_matrix(4, 30, 2.0, 80)
    e = oracle.s1_row_exponents(A)
    p = 5
    D = sp.digits_signed7(A, e, p, 1)
    assert np.abs(D).max() <= 127
    for i in range(4):
        for k in range(30):
            x = Fraction(float(A[i, k])) / Fraction(2) ** int(e[i])
            val = sum(Fraction(int(D[t, i, k])) / Fraction(2) ** (7 * (t + 1)) for t in range(p))
            assert abs(x - val) < Fraction(1, 2 ** (7 * p)) and (val == 0 or (val > 0) == (x > 0))


@pytest.mark.slow
def test_slice_formats_on_the_headline_distribution():
    """(u - 0.5) exp(g), K = 8192 (the headline workload's distribution and
    depth), 8 x 8 outputs, E_cw against double-double: the balanced digits
    meet 1e-13 at p = 7 and are far below native FP64 at p = 8, while the
    paper's format (and the signed 7-bit one, about as accurate here) needs
    p = 8 for 1e-13 and stays above native FP64 there.  Measured here:
    balanced 5.6e-15 / 2.0e-17, paper 5.2e-13 / 2.3e-15, signed 7-bit
    3.1e-13 / 2.6e-15 at p = 7 / 8; native 5.0e-16."""
    K = 8192
    A = synth.phi_matrix(8, K, 1.0, synth.seed_for(2, K, 1.0, synth.ROLE_A))
    B = synth.phi_matrix(K, 8, 1.0, synth.seed_for(2, K, 1.0, synth.ROLE_B))
    hi, lo = oracle.gemm_dd(A, B)
    native = metrics.e_cw(oracle.gemm_naive(A, B), hi, lo, A, B)
    err = {}
    for p in (7, 8):
        err["balanced", p] = metrics.e_cw(oracle.s1_dgemm(A, B, p), hi, lo, A, B)
        err["paper", p] = metrics.e_cw(sp.dgemm(A, B, p), hi, lo, A, B)
        err["signed7", p] = metrics.e_cw(sp.dgemm_signed7(A, B, p), hi, lo, A, B)
    print({k: "%.2g" % v for k, v in err.items()}, "native %.2g" % native)
    for p in (7, 8):
        assert err["balanced", p] * 10 < min(err["paper", p], err["signed7", p])
    assert err["balanced", 7] <= 1e-13 < err["paper", 7]
    assert err["paper", 8] <= 1e-13
    assert err["balanced", 8] < native < err["paper", 8]
