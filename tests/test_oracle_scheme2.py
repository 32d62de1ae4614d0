"""Pins of the CPU oracle's Scheme II (Sec. II-C.2, Eqs. 4-8) and 3M complex
form (Sec. IV-B, Eq. 16) against brute force, exact big-integer products,
the CRT's defining property and the paper's printed moduli."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from oracle import scheme2 as s2

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_rows(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([int(x) for x in line.split()])
    return rows


def test_moduli_start_as_printed_in_the_paper():
    printed = _golden_rows("paper_moduli.txt")[0]
    assert s2.moduli(len(printed)) == printed


def test_moduli_greedy_pairwise_coprime():
    ms = s2.moduli(20)
    assert all(m <= 256 for m in ms)
    for a in range(len(ms)):
        for b in range(a):
            assert math.gcd(ms[a], ms[b]) == 1
    # greedy: every skipped number between consecutive picks shares a factor
    for idx in range(1, len(ms)):
        for c in range(ms[idx] + 1, ms[idx - 1]):
            assert any(math.gcd(c, q) > 1 for q in ms[:idx])


def test_gemm_counts_table():
    for p, g1, g2 in _golden_rows("paper_counts.txt"):
        assert p * (p + 1) // 2 == g1
        assert g2 == p
        D = np.ones((p, 1, 1), np.int8) if p <= 8 else None
        if D is not None:
            Cd = oracle.s1_diagonals(D, D)[:, 0, 0]
            assert int(Cd.sum()) == g1 and Cd[0] == 1 and Cd[-1] == p


def test_crt_basis_property():
    """W_l = (P/m_l) q_l is 1 mod m_l and 0 mod every other modulus."""
    for s in (1, 3, 8, 16, 20):
        P, ms, W = s2.crt_constants(s)
        assert P == math.prod(ms)
        for l, w in enumerate(W):
            for k, m in enumerate(ms):
                assert w % m == (1 if k == l else 0)


def test_targets_satisfy_exactness_condition():
    for s in range(1, 21):
        P, _, _ = s2.crt_constants(s)
        ta, tb = s2.targets(s)
        assert 2 ** (ta + tb + 1) <= P  # 2 sum|a'||b'| < 2^(T_A+T_B+1) <= P


def test_smod_range_and_congruence():
    for m in (5, 7, 8, 9, 173, 255, 256):
        x = np.arange(-3 * m, 3 * m, dtype=np.int64)
        r = s2.smod(x, m)
        assert np.all((r - x) % m == 0)
        assert r.min() == -(m // 2) and r.max() == (m + 1) // 2 - 1


@pytest.mark.parametrize("ms", [[5, 7, 8, 9], [3, 4, 5], [256, 255, 253]])
def test_crt_brute_force(ms):
    """Every z in [-P/2, P/2) is the unique integer with its residues, and the
    CRT returns it (exhaustive for small P, sampled plus edges otherwise)."""
    P = math.prod(ms)
    if P <= 10000:
        zs = np.arange(-(P // 2), P - P // 2, dtype=np.int64)
        # uniqueness by enumeration
        keys = {tuple(int(s2.smod(int(z), m)) for m in ms) for z in zs}
        assert len(keys) == P
    else:
        rng = np.random.default_rng(0)
        zs = np.concatenate([rng.integers(-(P // 2), P - P // 2, 20000),
                             [-(P // 2), -(P // 2) + 1, -1, 0, 1, P - P // 2 - 1]]).astype(np.int64)
    Cl = [s2.smod(zs, m).astype(np.int8) for m in ms]
    got = s2.crt_for(Cl, ms)
    assert [int(v) for v in got] == [int(z) for z in zs]


def test_residues_crt_back_to_integers():
    rng = np.random.default_rng(3)
    for s in (8, 16):
        ta, _ = s2.targets(s)
        X = rng.integers(-(2 ** ta) + 1, 2 ** ta, size=(7, 9)).astype(np.float64)
        X = np.trunc(X)
        Cl = [s2.residues(X, m) for m in s2.moduli(s)]
        back = s2.crt(Cl, s)
        assert all(int(b) == int(x) for b, x in zip(back.ravel(), X.ravel()))


def test_scales_bound_norms_and_integerise_exactly():
    A = synth.phi_matrix(17, 64, 2.0, 9)
    A[4] = 0
    A[6] *= 1e-300
    ta, tb = s2.targets(14)
    sig, bad = s2.row_scales(A, ta)
    assert not bad.any()
    Ai = s2.integerise(A, sig, 1)
    for i in range(A.shape[0]):
        if not A[i].any():
            assert not Ai[i].any()
            continue
        # ||a_i||_2 2^sigma < 2^T_A, checked exactly
        nrm2 = sum(Fraction(float(v)) ** 2 for v in A[i]) * Fraction(4) ** int(sig[i])
        assert nrm2 < Fraction(4) ** ta
        for k in range(A.shape[1]):
            exact = Fraction(float(A[i, k])) * Fraction(2) ** int(sig[i])
            assert Ai[i, k] == math.trunc(exact)


@pytest.mark.parametrize("s", [6, 12, 16])
def test_s2_equals_plain_definition(s):
    """The CRT path reproduces RN(2^-sigma (A' B') 2^-tau) with an exact
    big-integer product, and the exactness condition holds on the input."""
    A = synth.phi_matrix(9, 31, 1.0, 50 + s)
    B = synth.phi_matrix(31, 11, 1.0, 60 + s)
    got, st = s2.s2_dgemm(A, B, s, return_parts=True)
    ref = s2.s2_exact_definition(A, B, s)
    assert np.array_equal(got, ref)
    P, _, _ = s2.crt_constants(s)
    big = np.vectorize(int, otypes=[object])
    absA = np.abs(big(st["Ai"].astype(object)))
    absB = np.abs(big(st["Bi"].astype(object)))
    assert (2 * (absA @ absB) < P).all()
    for ra, rb, m, cl in zip(st["RA"], st["RB"], st["ms"], st["Cl"]):
        prod = big(st["Ai"].astype(object)) @ big(st["Bi"].astype(object))
        assert ((prod - cl.astype(np.int64).astype(object)) % m == 0).all()


def test_s2_exact_for_small_integers():
    """Integer inputs that fit the bit budget come out exact."""
    rng = np.random.default_rng(4)
    A = rng.integers(-1000, 1000, size=(6, 12)).astype(np.float64)
    B = rng.integers(-1000, 1000, size=(12, 5)).astype(np.float64)
    assert np.array_equal(s2.s2_dgemm(A, B, 8), A @ B)


def test_s2_alpha_beta_and_nonfinite():
    A = synth.uniform_matrix(5, 8, 1)
    B = synth.uniform_matrix(8, 4, 2)
    C0 = synth.uniform_matrix(5, 4, 3)
    H = s2.s2_dgemm(A, B, 10)
    assert np.array_equal(s2.s2_dgemm(A, B, 10, alpha=2.0, beta=0.0, C=np.full((5, 4), np.nan)), 2 * H)
    got = s2.s2_dgemm(A, B, 10, alpha=0.5, beta=-3.0, C=C0)
    for i in range(5):
        for j in range(4):
            assert got[i, j] == float(Fraction(0.5) * Fraction(float(H[i, j])) + Fraction(float(-3.0 * C0[i, j])))
    B2 = B.copy()
    B2[3, 2] = np.inf
    C = s2.s2_dgemm(A, B2, 10)
    assert np.isnan(C[:, 2]).all() and not np.isnan(np.delete(C, 2, axis=1)).any()


def test_s2_error_falls_with_s():
    A = synth.phi_matrix(24, 128, 1.0, 70)
    B = synth.phi_matrix(128, 20, 1.0, 71)
    hi, lo = oracle.gemm_dd(A, B)
    errs = [oracle.metrics.e_cw(s2.s2_dgemm(A, B, s), hi, lo, A, B) for s in (8, 10, 12, 14, 16)]
    for a, b in zip(errs[:-1], errs[1:-1]):
        assert b < a / 64, errs  # two more moduli add about 15.7 bits
    assert errs[-1] < 2.0 ** -53, errs  # s = 16 reaches the FP64 rounding floor


# ----------------------------------------------------------------------- 3M

@pytest.mark.parametrize("s", [7, 14])
def test_3m_equals_exact_4m(s):
    """Modular 3M is exact: the same result as the 4M big-integer product."""
    A = synth.complex_phi_matrix(7, 19, 1.0, 80, 81)
    B = synth.complex_phi_matrix(19, 6, 1.0, 82, 83)
    got = s2.z3m_gemm(A, B, s)
    ref = s2.z3m_exact_definition(A, B, s)
    assert np.array_equal(got, ref)


def test_3m_cancellation_case():
    """re ~ im (where floating-point 3M cancels badly) is still exact."""
    rng = np.random.default_rng(8)
    X = rng.standard_normal((6, 15))
    A = X + 1j * (X * (1 + 2.0 ** -40))
    Y = rng.standard_normal((15, 5))
    B = Y + 1j * (Y * (1 - 2.0 ** -40))
    assert np.array_equal(s2.z3m_gemm(A, B, 16), s2.z3m_exact_definition(A, B, 16))
    hi, lo = oracle.zgemm_dd(A, B)
    assert oracle.metrics.e_cw(s2.z3m_gemm(A, B, 16), hi, lo, A, B) < 1e-15


def test_3m_sum_plane_and_exactness_condition():
    A = synth.complex_phi_matrix(5, 9, 2.0, 84, 85)
    B = synth.complex_phi_matrix(9, 4, 2.0, 86, 87)
    s = 12
    st = s2.z3m_prepare(A, B, s)
    P, _, _ = s2.crt_constants(s)
    big = np.vectorize(int, otypes=[object])
    u = np.abs(big(st["Are"].astype(object))) + np.abs(big(st["Aim"].astype(object)))
    v = np.abs(big(st["Bre"].astype(object))) + np.abs(big(st["Bim"].astype(object)))
    assert (2 * (u @ v) < P).all()
    for ((r_re, r_im, r_sum), (s_re, s_im, s_sum)), m in zip(st["planes"], st["ms"]):
        assert ((r_sum.astype(int) - r_re - r_im) % m == 0).all()
        assert ((s_sum.astype(int) - s_re - s_im) % m == 0).all()


def test_scale_formula_at_the_k_limit():
    """K = 2^22 entries of one exponent push the norm-bound sum S to 2^62 (the
    largest K the library takes for Scheme II keeps it below 2^63): nb =
    e + ceil((62 - 40) / 2) = e + 11, and the scaled row norm stays below
    2^T as the exactness condition needs (exact check in integers)."""
    K = 1 << 22
    ta, _ = s2.targets(16)
    A = np.full((1, K), -0.75)  # e = 0
    sig, _ = s2.row_scales(A, ta)
    assert int(sig[0]) == ta - 11
    # ||a||^2 4^sigma = K (3/4)^2 4^(ta - 11) < 4^ta  <=>  9 K < 16 4^11
    assert 9 * K < 16 * 4 ** 11
    # one entry twice as large moves e up by one and nb with it
    A[0, 5] = -1.5
    sig2, _ = s2.row_scales(A, ta)
    assert int(sig2[0]) == ta - 12


def test_entries_match_full_results():
    A = synth.phi_matrix(12, 40, 1.0, 90)
    B = synth.phi_matrix(40, 9, 1.0, 91)
    A[3, 2] = np.nan
    rows = np.array([0, 3, 11, 5, 7])
    cols = np.array([0, 4, 8, 2, 7])
    full = s2.s2_dgemm(A, B, 13)
    got = s2.s2_entries(A, B, 13, rows, cols)
    assert np.array_equal(np.isnan(got), np.isnan(full[rows, cols]))
    ok = ~np.isnan(got)
    assert np.array_equal(got[ok], full[rows, cols][ok])
    Z = synth.complex_phi_matrix(10, 30, 1.0, 92, 93)
    W = synth.complex_phi_matrix(30, 8, 1.0, 94, 95)
    fz = s2.z3m_gemm(Z, W, 11)
    assert np.array_equal(s2.z3m_entries(Z, W, 11, rows[[0, 2, 3, 4]] % 10, cols[[0, 2, 3, 4]] % 8),
                          fz[rows[[0, 2, 3, 4]] % 10, cols[[0, 2, 3, 4]] % 8])


# ------------------------------------------------ binary32 operands and results

def test_rn_f32_matches_numpy_and_the_c_oracle():
    """The rational rounding to binary32 equals numpy's correctly rounded
    binary64 -> binary32 conversion on exact binary64 values (ties,
    subnormals, overflow), and the C oracle's independent integer rounding."""
    from fractions import Fraction
    import random
    import oracle
    rng = random.Random(5)
    for _ in range(3000):
        x = np.float64(rng.uniform(1, 2)) * 2.0 ** rng.randrange(-160, 130)
        for v in (x, -x):
            with np.errstate(over="ignore"):  # the overflow to infinity is one of the cases
                want = np.float32(v)
            assert s2.rn_f32(Fraction(float(v))).tobytes() == want.tobytes(), v
    for z, E in [(1, -150), (3, -151), (2 ** 24 + 1, 0), (2 ** 24 - 1, 104), (7, -300)]:
        assert s2.scaled_round_f32(z, E).tobytes() == oracle.round_scaled_f32(z, E).tobytes()
    for _ in range(2000):
        z = rng.randrange(1, 2 ** rng.randrange(1, 120))
        E = rng.randrange(-300, 40)
        assert s2.scaled_round_f32(-z, E).tobytes() == oracle.round_scaled_f32(-z, E).tobytes()


def test_fmaf_single_rounding():
    """fmaf rounds a*b + c once: where binary64 holds a*b + c exactly, it is
    numpy's conversion of that binary64 value."""
    from fractions import Fraction
    rng = np.random.default_rng(8)
    n = 0
    for _ in range(3000):
        a, b, c = (np.float32(v) for v in rng.standard_normal(3) * 2.0 ** rng.integers(-20, 20, 3))
        exact = Fraction(float(a)) * Fraction(float(b)) + Fraction(float(c))
        d = np.float64(a) * np.float64(b) + np.float64(c)
        if Fraction(float(d)) == exact:
            n += 1
            assert s2._fmaf(a, b, c).tobytes() == np.float32(d).tobytes()
    assert n > 1000


def test_sgemm_and_cgemm_exact_for_small_integers():
    """Small integer operands are integerised without loss, so the binary32
    Scheme II and 3M results are the exact integer products (below 2^24)."""
    rng = np.random.default_rng(9)
    A = rng.integers(-100, 101, (7, 30)).astype(np.float32)
    B = rng.integers(-100, 101, (30, 6)).astype(np.float32)
    want = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float32)
    for s in (8, 12, 20):
        assert np.array_equal(s2.s2_sgemm(A, B, s), want)
    Ac = (A + 1j * rng.integers(-100, 101, A.shape)).astype(np.complex64)
    Bc = (B + 1j * rng.integers(-100, 101, B.shape)).astype(np.complex64)
    wre = Ac.real.astype(np.int64) @ Bc.real.astype(np.int64) - Ac.imag.astype(np.int64) @ Bc.imag.astype(np.int64)
    wim = Ac.real.astype(np.int64) @ Bc.imag.astype(np.int64) + Ac.imag.astype(np.int64) @ Bc.real.astype(np.int64)
    got = s2.z3m_cgemm(Ac, Bc, 10)
    assert np.array_equal(got.real, wre.astype(np.float32)) and np.array_equal(got.imag, wim.astype(np.float32))
