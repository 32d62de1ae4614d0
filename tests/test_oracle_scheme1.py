"""Pins of the CPU oracle's Scheme I (Sec. II-C.1, Eqs. 1-3) against facts that
do not come from the oracle itself: exact rational arithmetic, numpy's integer
matmul, Python's correctly rounded integer division, closed-form special cases
and the error trend the paper states (about one slice width of bits per
slice)."""
import math
import random
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth


def frac(x):
    return Fraction(float(x))


# --------------------------------------------------------------- exponents

def test_expo_brackets_value():
    vals = [1.0, 0.5, 0.75, 3.0, -7.9, 1e-300, 5e-324, 2.2250738585072014e-308,
            1.7976931348623157e308, -2.0 ** -1074, 2.0 ** 52 + 1]
    rng = np.random.default_rng(1)
    vals += list(rng.standard_normal(200) * 10.0 ** rng.integers(-300, 300, 200))
    for v in vals:
        e = oracle.expo(v)
        assert Fraction(2) ** (e - 1) <= abs(frac(v)) < Fraction(2) ** e, v


def test_row_and_col_exponents_are_the_max():
    A = synth.phi_matrix(37, 53, 2.0, 11)
    A[3, :] = 0.0
    e = oracle.s1_row_exponents(A)
    f = oracle.s1_col_exponents(A.T.copy())
    assert np.array_equal(e, f)
    for i in range(A.shape[0]):
        row = A[i]
        if not row.any():
            assert e[i] == oracle.ZERO_EXP
            continue
        assert np.all(np.abs(row) < 2.0 ** e[i])
        assert np.any(np.abs(row) >= 2.0 ** (e[i] - 1))
    A[5, 7] = np.inf
    assert oracle.s1_row_exponents(A)[5] == oracle.NONFINITE_EXP


# ------------------------------------------------------------------ digits

def _digit_sum(D, idx, p):
    """sum_t d_t 2^(-6-8t) as an exact fraction."""
    return sum(Fraction(int(D[(t,) + idx]), 2 ** (6 + 8 * t)) for t in range(p))


def _round_half_up(q: Fraction) -> int:
    return math.floor(q + Fraction(1, 2))


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6, 7, 8])
def test_slices_sum_back_exactly(p):
    """sum_t d_t 2^(-6-8t) equals x = a 2^-e rounded (half up) to 8p-2
    fraction bits; every slice fits a signed INT8 and the leading one |d_0| <= 64."""
    A = synth.phi_matrix(6, 40, 2.0, 100 + p)
    A[1, :6] = [2.0 ** -1070, -3e-310, 1e300, 0.0, -1.0, -1e-300]
    A[2, :4] = [1.0 - 2.0 ** -53, -2.0 ** -1074, -5e-324, -(1.0 - 2.0 ** -40)]
    e = oracle.s1_row_exponents(A)
    D = oracle.s1_digits_a(A, e, p)
    assert D.dtype == np.int8
    assert np.abs(D[0].astype(int)).max() <= 64
    for i in range(A.shape[0]):
        for k in range(A.shape[1]):
            x = frac(A[i, k]) / Fraction(2) ** int(e[i])
            assert abs(x) < 1
            X = _round_half_up(x * 2 ** (8 * p - 2))
            assert _digit_sum(D, (i, k), p) == Fraction(X, 2 ** (8 * p - 2)), (i, k)
            assert abs(_digit_sum(D, (i, k), p) - x) <= Fraction(1, 2 ** (8 * p - 1))


def test_slices_exact_for_short_mantissas():
    """An entry with at most 8p-2 fraction bits below the row exponent is
    represented exactly."""
    rng = np.random.default_rng(5)
    p = 3
    m = rng.integers(-(2 ** 22) + 1, 2 ** 22, size=(4, 30))
    A = np.ldexp(m.astype(np.float64), -22)
    A[:, 0] = 1.0 - 2.0 ** -22  # pins the row exponent at 0
    e = oracle.s1_row_exponents(A)
    assert np.all(e == 0)
    D = oracle.s1_digits_a(A, e, p)
    for i in range(4):
        for k in range(30):
            assert _digit_sum(D, (i, k), p) == frac(A[i, k])


def test_digit_special_cases():
    p = 4
    # x close to +-1 rounds to X = +-2^(8p-2): leading digit +-64, rest 0
    A = np.array([[1.0 - 2.0 ** -40, -(1.0 - 2.0 ** -40)]])
    D = oracle.s1_digits_a(A, oracle.s1_row_exponents(A), p)
    assert list(D[:, 0, 0]) == [64, 0, 0, 0]
    assert list(D[:, 0, 1]) == [-64, 0, 0, 0]
    # X = 2^(8p-2) - 1 = 63*256^3 + 255*256^2 + 255*256 + 255 -> balanced 64, 0, 0, -1
    A = np.array([[1.0 - 2.0 ** -30]])
    D = oracle.s1_digits_a(A, oracle.s1_row_exponents(A), p)
    assert list(D[:, 0, 0]) == [64, 0, 0, -1]
    # X = 128 -> trailing digit -128 with a carry of one into the next digit
    A = np.array([[0.5, 2.0 ** -23]])
    D = oracle.s1_digits_a(A, oracle.s1_row_exponents(A), p)
    assert list(D[:, 0, 1]) == [0, 0, 1, -128]
    # tiny entries round to zero; exact halves of the last place round up
    A = np.array([[0.5, -2.0 ** -200, 2.0 ** -31, -2.0 ** -31]])
    D = oracle.s1_digits_a(A, oracle.s1_row_exponents(A), p)
    assert not D[:, 0, 1].any()
    assert list(D[:, 0, 2]) == [0, 0, 0, 1] and list(D[:, 0, 3]) == [0, 0, 0, 0]
    # x = 2^(-6-8t) -> one-hot at slice t (row exponent fixed at 0 by 0.5)
    for t in range(p):
        A = np.array([[0.5, 2.0 ** (-6 - 8 * t)]])
        D = oracle.s1_digits_a(A, oracle.s1_row_exponents(A), p)
        expect = np.zeros(p, np.int8)
        expect[t] = 1
        assert np.array_equal(D[:, 0, 1], expect)
        assert D[0, 0, 0] == 32 and not D[1:, 0, 0].any()


def test_b_digits_match_a_digits_of_transpose():
    B = synth.phi_matrix(21, 17, 1.0, 8)
    f = oracle.s1_col_exponents(B)
    E = oracle.s1_digits_b(B, f, 5)
    D = oracle.s1_digits_a(B.T.copy(), f, 5)
    assert np.array_equal(E, D.transpose(0, 2, 1))


def test_k_split_bound():
    """The longest overflow-free K run: (p-1) 2^14 k (or 2^12 k for p = 1)
    stays below 2^31."""
    for p in range(1, 9):
        k = oracle.k_split_s1(p)
        assert k % 32 == 0
        per_k = max(2 ** 12, (p - 1) * 2 ** 14)
        assert per_k * k < 2 ** 31 <= per_k * (k + 32)
    # every diagonal at the worst-case digits reaches the stated per-k bound
    p = 8
    D = np.full((p, 1, 1), -128, np.int8)
    D[0] = -64
    Cd = oracle.s1_diagonals(D, D)[:, 0, 0]
    assert max(abs(int(c)) for c in Cd) == (p - 1) * 2 ** 14


# --------------------------------------------------------------- diagonals

@pytest.mark.parametrize("p", [1, 3, 8])
def test_diagonals_equal_integer_matmul(p):
    """Eq. 2 against numpy's int64 matmul of the slice planes."""
    rng = np.random.default_rng(p)
    M, N, K = 13, 11, 29
    D = rng.integers(-128, 128, size=(p, M, K)).astype(np.int8)
    E = rng.integers(-128, 128, size=(p, K, N)).astype(np.int8)
    Cd = oracle.s1_diagonals(D, E)
    for d in range(p):
        ref = sum(D[t].astype(np.int64) @ E[d - t].astype(np.int64) for t in range(d + 1))
        assert np.array_equal(Cd[d], ref)


def test_diagonal_index_is_sum_of_slice_indices():
    """A single one-hot product A'_t B'_u lands only in accumulator t+u, and
    accumulator d collects d+1 slice pairs (Sec. II-C.1: C_0 one product,
    C_(p-1) p products)."""
    p = 5
    for t in range(p):
        for u in range(p):
            D = np.zeros((p, 1, 1), np.int8)
            E = np.zeros((p, 1, 1), np.int8)
            D[t] = 1
            E[u] = 1
            Cd = oracle.s1_diagonals(D, E)[:, 0, 0]
            expect = np.zeros(p, np.int64)
            if t + u < p:
                expect[t + u] = 1
            assert np.array_equal(Cd, expect)
    D = np.ones((p, 1, 1), np.int8)
    Cd = oracle.s1_diagonals(D, D)[:, 0, 0]
    assert list(Cd) == [d + 1 for d in range(p)]
    assert sum(Cd) == p * (p + 1) // 2


# ---------------------------------------------------------------- rounding

def _py_round(Z, E):
    if E >= 0:
        try:
            return float(Z << E)
        except OverflowError:
            return math.copysign(math.inf, Z)
    return Z / (1 << -E)


def test_round_scaled_matches_correct_rounding():
    rnd = random.Random(3)
    cases = [(0, 0), (1, -1074), (1, -1075), (3, -1076), (2 ** 53 + 1, 0),
             (2 ** 53 + 3, 0), (-(2 ** 53 + 1), 0), (2 ** 54 + 2, -1), (2 ** 100 + 2 ** 47, -100),
             (2 ** 100 + 2 ** 47 + 1, -100), ((2 ** 53 - 1) << 60, 1024 - 113),
             ((2 ** 53 - 1) << 60, 1024 - 112), (2 ** 126, -1200), (2 ** 127 - 1, -1201),
             (2 ** 126 + 1, -1201), (5, -1077), (7, -1076), ((1 << 120) + 1, -1194)]
    for _ in range(3000):
        n = rnd.randint(1, 126)
        Z = rnd.getrandbits(n) * rnd.choice([1, -1])
        if rnd.random() < 0.3 and n > 54:  # force exact ties
            Z = (Z >> (n - 54) << (n - 54)) | (1 << (n - 55))
        E = rnd.choice([rnd.randint(-1250, -1000), rnd.randint(-200, 100), rnd.randint(900, 1000)])
        cases.append((Z, E))
    for Z, E in cases:
        got = oracle.round_scaled(Z, E)
        ref = _py_round(Z, E)
        assert got == ref or (math.isinf(got) and math.isinf(ref) and got == ref), (Z, E, got, ref)


# ------------------------------------------------------------ whole scheme

def _exact_product(A, B):
    M, K = A.shape
    N = B.shape[1]
    FA = [[frac(A[i, k]) for k in range(K)] for i in range(M)]
    FB = [[frac(B[k, j]) for j in range(N)] for k in range(K)]
    return [[sum(FA[i][k] * FB[k][j] for k in range(K)) for j in range(N)] for i in range(M)]


@pytest.mark.parametrize("ra,rb,p", [(1, 1, 1), (2, 3, 4), (3, 3, 5), (4, 4, 7), (2, 1, 2)])
def test_exact_when_all_digit_pairs_fit(ra, rb, p):
    """If A's entries need ra digits and B's rb with ra + rb - 1 <= p, no
    slice pair is dropped, so the result is RN(exact A B).  (ra = rb = p = 1 is
    a plain INT8 GEMM.)"""
    rng = np.random.default_rng(100 * ra + rb)
    M, N, K = 5, 6, 23
    ba, bb = 8 * ra - 2, 8 * rb - 2
    ma = rng.integers(-(2 ** ba) + 1, 2 ** ba, size=(M, K))
    mb = rng.integers(-(2 ** bb) + 1, 2 ** bb, size=(K, N))
    ma[:, 0] = 2 ** ba - 1  # row maximum fixes the row exponent
    mb[0, :] = -(2 ** bb) + 1
    A = np.ldexp(ma.astype(np.float64), rng.integers(-30, 30, size=(M, 1)))
    B = np.ldexp(mb.astype(np.float64), rng.integers(-30, 30, size=(1, N)))
    C = oracle.s1_dgemm(A, B, p)
    X = _exact_product(A, B)
    for i in range(M):
        for j in range(N):
            assert C[i, j] == float(X[i][j]), (i, j)


def test_truncated_digits_drop_only_low_pairs():
    """With p too small the result differs from the exact product by less
    than the dropped-weight bound: per term, rounding residues below
    2^-(8p-1) of each scale plus the dropped pairs (below p 2^-(8p-2))."""
    A = synth.phi_matrix(8, 16, 0.5, 21)
    B = synth.phi_matrix(16, 9, 0.5, 22)
    p = 2
    C = oracle.s1_dgemm(A, B, p)
    X = _exact_product(A, B)
    e = oracle.s1_row_exponents(A)
    f = oracle.s1_col_exponents(B)
    K = A.shape[1]
    for i in range(8):
        for j in range(9):
            scale = Fraction(2) ** (int(e[i]) + int(f[j]))
            err = abs(frac(C[i, j]) - X[i][j])
            bound = K * (p + 2) * Fraction(1, 2 ** (8 * p - 2)) * scale + abs(X[i][j]) * Fraction(1, 2 ** 52)
            assert err <= bound


def test_alpha_beta_and_edge_shapes():
    A = synth.uniform_matrix(7, 5, 1)
    B = synth.uniform_matrix(5, 3, 2)
    C0 = synth.uniform_matrix(7, 3, 3)
    H = oracle.s1_dgemm(A, B, 4)
    # beta == 0 must not read C (NaN in C stays out of the result)
    Cn = np.full((7, 3), np.nan)
    assert np.array_equal(oracle.s1_dgemm(A, B, 4, alpha=2.0, beta=0.0, C=Cn), 2.0 * H)
    got = oracle.s1_dgemm(A, B, 4, alpha=-1.5, beta=0.25, C=C0)
    for i in range(7):
        for j in range(3):
            ref = float(Fraction(-1.5) * frac(H[i, j]) + frac(0.25 * C0[i, j]))
            assert got[i, j] == ref
    # K = 0 gives zeros; zero rows/columns give exact zeros
    Z = oracle.s1_dgemm(np.zeros((3, 0)), np.zeros((0, 4)), 3)
    assert Z.shape == (3, 4) and not Z.any()
    A2 = A.copy()
    A2[2] = 0
    assert not oracle.s1_dgemm(A2, B, 4)[2].any()
    A2[4, 1] = np.nan
    C = oracle.s1_dgemm(A2, B, 4)
    assert np.isnan(C[4]).all() and not np.isnan(np.delete(C, 4, axis=0)).any()


def test_entries_match_full_result():
    A = synth.phi_matrix(40, 70, 1.0, 31)
    B = synth.phi_matrix(70, 50, 1.0, 32)
    p = 6
    full = oracle.s1_dgemm(A, B, p)
    rng = np.random.default_rng(0)
    rows = rng.integers(0, 40, 60)
    cols = rng.integers(0, 50, 60)
    assert np.array_equal(oracle.s1_entries(A, B, p, rows, cols), full[rows, cols])


def test_error_falls_to_fp64_level_as_p_grows():
    """About 8 bits per extra slice until the FP64 floor (Sec. II-C.1)."""
    A = synth.phi_matrix(48, 256, 1.0, 41)
    B = synth.phi_matrix(256, 40, 1.0, 42)
    hi, lo = oracle.gemm_dd(A, B)
    errs = [oracle.metrics.e_cw(oracle.s1_dgemm(A, B, p), hi, lo, A, B) for p in range(1, 9)]
    assert errs[1] < errs[0] / 8, errs  # the leading slice carries 6 bits only
    for p in range(2, 7):
        assert errs[p] < errs[p - 1] / 64, errs  # at least 6 bits per further slice
    nat = oracle.metrics.e_cw(oracle.gemm_naive(A, B), hi, lo, A, B)
    assert errs[6] < 1e-13, errs  # the 1e-13 gate from p = 7
    assert errs[7] <= 2 * nat, (errs, nat)  # within 2x of native FP64 at p = 8


# ------------------------------------------------ binary32 operands and result

def test_round_scaled_f32_matches_numpy_conversion():
    """For |Z| < 2^53, Z 2^E is an exact binary64 value and numpy's
    binary64 -> binary32 conversion is a correctly rounded one (ties to even,
    gradual underflow, overflow to infinity): the oracle's direct rounding
    must agree, including ties and the subnormal and overflow edges."""
    rng = random.Random(11)
    cases = [(1, -149), (1, -150), (3, -151), (2 ** 24 + 1, 0), (2 ** 24 + 3, 0), (2 ** 25 - 1, 103),
             ((2 ** 24 - 1) * 2, 103), (2 ** 24 - 1, 104), (5, -152), (2 ** 52 + 1, -200)]
    for _ in range(3000):
        z = rng.randrange(1, 2 ** rng.randrange(1, 53))
        cases.append((z, rng.randrange(-230, 110)))
    for z, E in cases:
        for sz in (z, -z):
            with np.errstate(over="ignore"):  # the overflow to infinity is one of the cases
                want = np.float32(np.ldexp(np.float64(sz), E))
            got = oracle.round_scaled_f32(sz, E)
            assert got.tobytes() == want.tobytes(), (sz, E, got, want)


def test_sgemm_exact_for_small_integers():
    """Integer entries of at most 7 bits occupy the two leading digits of the
    balanced format (slice 0 carries 6 bits and the sign), so from p = 3 on
    every digit pair is kept; sums below 2^24 are exact binary32 values, so
    the emulated SGEMM is the exact integer product.  Zero rows and columns
    give zeros and a non-finite entry gives NaN in its row (A) and column
    (B)."""
    rng = np.random.default_rng(3)
    for p in (3, 5, 8):
        M, N, K = 9, 7, 40
        A = rng.integers(-127, 128, (M, K)).astype(np.float32)
        B = rng.integers(-127, 128, (K, N)).astype(np.float32)
        A[2] = 0
        B[:, 3] = 0
        want = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float32)
        assert np.array_equal(oracle.s1_sgemm(A, B, p), want)
        assert np.array_equal(oracle.s1_sgemm(A, B, p, alpha=2.0), 2 * want)
        A[4, 5] = np.inf
        B[6, 1] = np.nan
        got = oracle.s1_sgemm(A, B, p)
        bad = np.zeros((M, N), bool)
        bad[4, :] = True
        bad[:, 1] = True
        assert np.isnan(got[bad]).all() and np.array_equal(got[~bad], want[~bad])


def test_sgemm_is_the_binary64_result_rounded_once():
    """The binary32 result is the exact Z 2^E rounded once; rounding the
    binary64 path's result again can differ only by double rounding, i.e. by
    at most one binary32 ulp, and only rarely."""
    A = synth.phi_matrix(60, 90, 1.0, 21).astype(np.float32)
    B = synth.phi_matrix(90, 50, 1.0, 22).astype(np.float32)
    for p in (1, 2, 3, 4, 6):
        got = oracle.s1_sgemm(A, B, p)
        twice = oracle.s1_dgemm(A.astype(np.float64), B.astype(np.float64), p).astype(np.float32)
        diff = got.view(np.int32).astype(np.int64) - twice.view(np.int32).astype(np.int64)
        assert np.abs(diff).max() <= 1 and np.count_nonzero(diff) <= got.size // 100, p
