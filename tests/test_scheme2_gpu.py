"""Scheme II (real) and 3M ZGEMM on the GPU against the CPU oracle, through
the C ABI.  Bit-exact: scale exponents, residue planes (Eq. 5), the per-modulus
INT8 output residues (Eqs. 6-7, Eq. 16) and the FP64 / complex128 outputs
after the CRT (Eq. 8) and one rounding."""
import numpy as np
import pytest

import oracle
import paper_2606_25453_amd as ozk
import synth
from oracle import scheme2 as s2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = ozk.Context(0)
    yield c
    c.close()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rp(n):
    return (n + 255) // 256 * 256


def kp(k):
    return (k + 31) // 32 * 32


def planes_real(packed, s, rows, K):
    """[s][c][r][32] -> [s][Rp][Kp]"""
    return host(packed)[: s * rp(rows) * kp(K)].reshape(s, kp(K) // 32, rp(rows), 32).transpose(0, 2, 1, 3).reshape(
        s, rp(rows), kp(K))


def planes_cplx(packed, s, rows, K):
    """[s][c][q][r][32] -> [s][q][Rp][Kp]"""
    return host(packed)[: 3 * s * rp(rows) * kp(K)].reshape(s, kp(K) // 32, 3, rp(rows), 32).transpose(
        0, 2, 3, 1, 4).reshape(s, 3, rp(rows), kp(K))


@pytest.mark.parametrize("s", [1, 8, 13, 16, 20])
@pytest.mark.parametrize("shape", [(37, 70), (300, 129)])
def test_split_rows_real(ctx, s, shape):
    rows, K = shape
    X = synth.phi_matrix(rows, K, 2.0, 500 + s)
    X[min(2, rows - 1)] = 0
    X[min(4, rows - 1)] *= 1e-290
    X[min(5, rows - 1), :3] = [5e-324, -1e-310, 2.0 ** -1060]  # subnormals beside normal entries
    X[min(6, rows - 1)] = np.ldexp(X[min(6, rows - 1)], -1040)  # a row of subnormals
    sig, packed = ozk.ozk_s2_split_rows(ctx, s, dev(X))
    ta, _ = s2.targets(s)
    ref_sig, _ = s2.row_scales(X, ta)
    assert np.array_equal(host(sig)[:rows], ref_sig)
    R = planes_real(packed, s, rows, K)
    Xi = s2.integerise(X, ref_sig, 1)
    for l, m in enumerate(s2.moduli(s)):
        assert np.array_equal(R[l, :rows, :K], s2.residues(Xi, m)), l
    assert not R[:, rows:, :].any() and not R[:, :, K:].any()


@pytest.mark.parametrize("s", [2, 14, 20])
@pytest.mark.parametrize("shape", [(70, 37), (129, 300), (700, 77), (1100, 300)])
def test_split_cols_real(ctx, s, shape):
    K, cols = shape
    X = synth.phi_matrix(K, cols, 2.0, 600 + s)
    X[:, min(3, cols - 1)] = 0
    X[:, min(4, cols - 1)] *= 1e-300  # with long K the scales take the split-over-K path
    X[: K // 3, min(5, cols - 1)] *= 1e-30
    tau, packed = ozk.ozk_s2_split_cols(ctx, s, dev(X))
    _, tb = s2.targets(s)
    ref_tau, _ = s2.col_scales(X, tb)
    assert np.array_equal(host(tau)[:cols], ref_tau)
    R = planes_real(packed, s, cols, K)
    Xi = s2.integerise(X, ref_tau, 0)
    for l, m in enumerate(s2.moduli(s)):
        assert np.array_equal(R[l, :cols, :K], s2.residues(Xi, m).T), l
    assert not R[:, cols:, :].any() and not R[:, :, K:].any()


@pytest.mark.parametrize("s,K", [(5, 100), (16, 100), (20, 100), (16, 777)])
def test_split_complex(ctx, s, K):
    rows = 45
    X = synth.complex_phi_matrix(rows, K, 1.0, 700 + s, 710 + s)
    X[3] = X[3].real  # imaginary part zero in one row
    sig, packed = ozk.ozk_s2_split_rows(ctx, s, dev(X), complex_planes=1)
    Y = synth.complex_phi_matrix(K, rows, 1.0, 720 + s, 730 + s)
    tau, packedb = ozk.ozk_s2_split_cols(ctx, s, dev(Y), complex_planes=1)
    st = s2.z3m_prepare(X, Y, s)
    assert np.array_equal(host(sig)[:rows], st["sig"])
    assert np.array_equal(host(tau)[:rows], st["tau"])
    R = planes_cplx(packed, s, rows, K)
    S = planes_cplx(packedb, s, rows, K)
    for l in range(s):
        (r_re, r_im, r_sum), (s_re, s_im, s_sum) = st["planes"][l]
        assert np.array_equal(R[l, 0, :rows, :K], r_re)
        assert np.array_equal(R[l, 1, :rows, :K], r_im)
        assert np.array_equal(R[l, 2, :rows, :K], r_sum)
        assert np.array_equal(S[l, 0, :rows, :K], s_re.T)
        assert np.array_equal(S[l, 2, :rows, :K], s_sum.T)


@pytest.mark.parametrize("s", [3, 16])
@pytest.mark.parametrize("shape", [(63, 65, 127), (129, 257, 95), (61, 44, 90)])
def test_gemm_mod_residues_bit_exact(ctx, s, shape):
    # (61, 44, 90): N a multiple of 4, so the residues leave the GEMM as 4-byte
    # words transposed across lane quads; M leaves a partial group of rows
    M, N, K = shape
    A = synth.phi_matrix(M, K, 1.0, 800 + s)
    B = synth.phi_matrix(K, N, 1.0, 810 + s)
    sig, pa = ozk.ozk_s2_split_rows(ctx, s, dev(A))
    tau, pb = ozk.ozk_s2_split_cols(ctx, s, dev(B))
    Cres = host(ozk.ozk_s2_gemm_mod(ctx, s, M, N, K, pa, pb))
    st = s2.s2_prepare(A, B, s)
    for l, m in enumerate(st["ms"]):
        assert np.array_equal(Cres[l], s2.modular_product(st["RA"][l], st["RB"][l], m)), l


@pytest.mark.parametrize("M,N", [(70, 90), (61, 44)])
def test_gemm_mod_3m_residues_bit_exact(ctx, M, N):
    # (61, 44): the 4-byte transposed residue stores (N a multiple of 4)
    s, K = 9, 110
    A = synth.complex_phi_matrix(M, K, 1.0, 900, 901)
    B = synth.complex_phi_matrix(K, N, 1.0, 902, 903)
    _, pa = ozk.ozk_s2_split_rows(ctx, s, dev(A), complex_planes=1)
    _, pb = ozk.ozk_s2_split_cols(ctx, s, dev(B), complex_planes=1)
    Cres = host(ozk.ozk_s2_gemm_mod(ctx, s, M, N, K, pa, pb, complex_planes=1)).reshape(s, 2, M, N)
    st = s2.z3m_prepare(A, B, s)
    for l, m in enumerate(st["ms"]):
        re, im = s2.z3m_modular(st["planes"][l][0], st["planes"][l][1], m)
        assert np.array_equal(Cres[l, 0], re) and np.array_equal(Cres[l, 1], im), l


@pytest.mark.parametrize("s", [1, 6, 8, 12, 14, 16, 18, 20])
@pytest.mark.parametrize("shape", [(1, 1, 1), (63, 65, 127), (129, 130, 95), (200, 64, 300)])
def test_dgemm_scheme2_bit_exact(ctx, s, shape):
    M, N, K = shape
    A = synth.phi_matrix(M, K, 1.0, 1000 + s + M)
    B = synth.phi_matrix(K, N, 1.0, 1100 + s + N)
    C = host(ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME2, s, dev(A), dev(B)))
    assert np.array_equal(C, s2.s2_dgemm(A, B, s))



@pytest.mark.parametrize("s", list(range(1, 21)))
@pytest.mark.parametrize("cplx", [False, True])
def test_crt_every_modulus_count(ctx, s, cplx):
    """The CRT has one straight-line body per modulus count (chosen by a
    uniform branch inside the kernel of the count's limb count): every count
    1..20, real and 3M, against the oracle on a ragged shape."""
    M, N, K = 37, 45, 70
    if cplx:
        A = synth.complex_phi_matrix(M, K, 1.0, 2000 + s, 2100 + s)
        B = synth.complex_phi_matrix(K, N, 1.0, 2200 + s, 2300 + s)
        C = host(ozk.ozk_zgemm_3m(ctx, s, dev(A), dev(B)))
        assert np.array_equal(C, s2.z3m_gemm(A, B, s))
    else:
        A = synth.phi_matrix(M, K, 1.0, 2400 + s)
        B = synth.phi_matrix(K, N, 1.0, 2500 + s)
        C = host(ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME2, s, dev(A), dev(B)))
        assert np.array_equal(C, s2.s2_dgemm(A, B, s))

@pytest.mark.parametrize("s", [1, 2, 7, 11, 14, 15, 16, 20])
@pytest.mark.parametrize("cplx", [False, True])
def test_crt_near_half_multiples_of_p(ctx, s, cplx):
    """Residue sets whose CRT value Z lies at and next to -P/2 and P/2 - 1
    (the ends of the symmetric range, where the sum V is at or next to a
    half-multiple of P: the binary64 quotient estimate cannot settle q there
    and the exact steps decide), at 0 and +-1, and random ones, through the
    CRT entry point: Z rebuilt by the oracle's CRT (Eq. 8) must equal the
    chosen values, and the outputs its rounding (sigma, tau in [30, 60])."""
    ms = s2.moduli(s)
    P = 1
    for m in ms:
        P *= m
    half = P // 2
    rng = np.random.default_rng(s)
    M, N = 6, 7
    def targets(flip):
        t = [-half, -half + 1, -half + 2, half - 1, half - 2, half - 3, 0, 1, -1, half // 3, -(half // 7)]
        t = [max(-half, min(half - 1, v)) for v in t]
        t += [int(rng.integers(-2 ** 62, 2 ** 62)) * (half // 2 ** 62 + 1) % P - half for _ in range(M * N - len(t))]
        z = np.array(t, dtype=object).reshape(M, N)
        return -z - 1 if flip else z  # -z - 1 keeps [-P/2, P/2)
    Zt = [targets(False)] + ([targets(True)] if cplx else [])
    planes = []
    for l, m in enumerate(ms):
        for z in Zt:
            planes.append(np.array([[s2.smod(int(v) % m, m) for v in row] for row in z], np.int8))
    res = np.stack(planes)  # [l][re, im][M][N]
    sig = rng.integers(30, 61, M).astype(np.int32)
    tau = rng.integers(30, 61, N).astype(np.int32)
    want = []
    for q, z in enumerate(Zt):
        Z = s2.crt([res[len(Zt) * l + q] for l in range(s)], s)
        assert np.array_equal(Z, z)  # the construction itself
        want.append(np.array([[s2.scaled_round(int(Z[i, j]), -int(sig[i]) - int(tau[j])) for j in range(N)]
                              for i in range(M)]))
    C = torch.empty((M, N), dtype=torch.complex128 if cplx else torch.float64, device="cuda:0")
    got = host(ozk.ozk_s2_crt(ctx, s, M, N, dev(res), dev(sig), dev(tau), C, complex_planes=int(cplx)))
    if cplx:
        assert np.array_equal(got.real, want[0]) and np.array_equal(got.imag, want[1])
    else:
        assert np.array_equal(got, want[0])


@pytest.mark.parametrize("cplx", [False, True])
def test_column_scales_wide_short_k(ctx, cplx):
    """Very many columns with short K: more column blocks than can hold their
    exponent caches on the GPU at once, so the scales take the two-pass
    column kernel; sampled columns (a column's scale depends on that column
    alone) against the oracle, and the single-read path on a narrow slice of
    the same B against the oracle too."""
    s, M, K, N = 4, 20, 256, 65536
    rng = np.random.default_rng(5)
    if cplx:
        A = synth.complex_phi_matrix(M, K, 1.0, 401, 402)
        B = synth.complex_phi_matrix(K, N, 1.0, 403, 404)
    else:
        A = synth.phi_matrix(M, K, 1.0, 401)
        B = synth.phi_matrix(K, N, 1.0, 403)
    B[::5, 7] = 0
    rows = np.sort(rng.choice(M, size=5, replace=False))
    cols = np.unique(np.concatenate([[7, N - 1], rng.choice(N, size=8, replace=False)]))
    call = (lambda a, b: ozk.ozk_zgemm_3m(ctx, s, a, b)) if cplx else \
        (lambda a, b: ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME2, s, a, b))
    ref_of = (lambda a, b: s2.z3m_gemm(a, b, s)) if cplx else (lambda a, b: s2.s2_dgemm(a, b, s))
    got = host(call(dev(A), dev(B)))
    assert np.array_equal(got[np.ix_(rows, cols)], ref_of(A[rows], B[:, cols]))
    narrow = np.ascontiguousarray(B[:, :300])
    got_n = host(call(dev(A), dev(narrow)))
    assert np.array_equal(got_n, got[:, :300])
    assert np.array_equal(got_n[rows], ref_of(A[rows], narrow))


def test_scheme2_alpha_beta_edges(ctx):
    s, M, N, K = 14, 40, 30, 50
    A = synth.phi_matrix(M, K, 1.0, 1)
    B = synth.phi_matrix(K, N, 1.0, 2)
    C0 = synth.phi_matrix(M, N, 1.0, 3)
    A[0] = 0
    A[1] *= 1e-300
    A[2] *= 1e300
    A[3, 4] = np.inf
    A[4] *= 1e-160  # with B[:, 8] below: products in the subnormal range
    A[5, :4] = [5e-324, -1e-310, 0.0, 2.0 ** -1060]
    B[:, 5] = 0
    B[7, 6] = np.nan
    B[:, 8] *= 1e-160
    B[:, 9] *= 1e10  # with A[2]: products past the largest double
    got = host(ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME2, s, dev(A), dev(B), C=dev(C0), alpha=-1.5, beta=0.5))
    ref = s2.s2_dgemm(A, B, s, alpha=-1.5, beta=0.5, C=C0)
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    ok = ~np.isnan(ref)
    assert np.array_equal(got[ok], ref[ok])
    assert np.isnan(got[3]).all() and np.isnan(got[:, 6]).all()
    # without alpha/beta the subnormal (row 4, column 8) and infinite (2, 9) products show directly
    got0 = host(ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME2, s, dev(A), dev(B)))
    ref0 = s2.s2_dgemm(A, B, s)
    ok0 = ~np.isnan(ref0)
    assert np.array_equal(np.isnan(got0), np.isnan(ref0)) and np.array_equal(got0[ok0], ref0[ok0])
    assert 0 < abs(ref0[4, 8]) < np.finfo(np.float64).tiny and np.isinf(ref0[2, 9])


@pytest.mark.parametrize("s", [4, 11, 16])
@pytest.mark.parametrize("shape", [(1, 1, 1), (63, 65, 70), (130, 40, 96)])
def test_zgemm_3m_bit_exact(ctx, s, shape):
    M, N, K = shape
    A = synth.complex_phi_matrix(M, K, 1.0, 1200 + s, 1201 + s)
    B = synth.complex_phi_matrix(K, N, 1.0, 1202 + s, 1203 + s)
    C = host(ozk.ozk_zgemm_3m(ctx, s, dev(A), dev(B)))
    assert np.array_equal(C, s2.z3m_gemm(A, B, s))


def test_zgemm_3m_alpha_beta_and_cancellation(ctx):
    s, M, N, K = 16, 30, 20, 40
    rng = np.random.default_rng(5)
    X = rng.standard_normal((M, K))
    A = X + 1j * X * (1 + 2.0 ** -40)  # re ~ im
    B = synth.complex_phi_matrix(K, N, 1.0, 1300, 1301)
    C0 = synth.complex_phi_matrix(M, N, 1.0, 1302, 1303)
    al, be = 0.5 - 2j, -1 + 0.25j
    got = host(ozk.ozk_zgemm_3m(ctx, s, dev(A), dev(B), C=dev(C0), alpha=al, beta=be))
    assert np.array_equal(got, s2.z3m_gemm(A, B, s, alpha=al, beta=be, C=C0))
    got0 = host(ozk.ozk_zgemm_3m(ctx, s, dev(A), dev(B), C=dev(np.full((M, N), np.nan + 0j))))
    assert np.array_equal(got0, s2.z3m_gemm(A, B, s))


def test_empty_and_invalid(ctx):
    for (M, N, K) in [(0, 4, 3), (4, 0, 3), (4, 3, 0)]:
        C = dev(np.full((M, N), 5.0))
        ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME2, 10, dev(np.ones((M, K))), dev(np.ones((K, N))), C=C)
        assert np.array_equal(host(C), np.zeros((M, N)))
    A = dev(np.ones((4, 4)))
    for bad in (0, 21):
        with pytest.raises(ozk.OzkError) as ei:
            ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME2, bad, A, A)
        assert ei.value.status == ozk.OZK_ERR_UNSUPPORTED


@pytest.mark.parametrize("n,s", [(4096, 14), (4096, 16)])
def test_large_scheme2_sampled(ctx, n, s):
    A = synth.phi_matrix(n, n, 1.0, synth.seed_for(3, n, 1.0, synth.ROLE_A))
    B = synth.phi_matrix(n, n, 1.0, synth.seed_for(3, n, 1.0, synth.ROLE_B))
    a, b = dev(A), dev(B)
    C = host(ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME2, s, a, b))
    rng = np.random.default_rng(n + s)
    rows = np.concatenate([rng.integers(0, n, 40), [0, n - 1]])
    cols = np.concatenate([rng.integers(0, n, 40), [n - 1, 0]])
    assert np.array_equal(C[rows, cols], s2.s2_entries(A, B, s, rows, cols))
    ri = rng.choice(n, 8, replace=False)
    ci = rng.choice(n, 8, replace=False)
    hi, lo = oracle.gemm_dd(A[ri], B[:, ci])
    err = oracle.metrics.e_cw(C[np.ix_(ri, ci)], hi, lo, A[ri], B[:, ci])
    nat = host(torch.matmul(a, b))[np.ix_(ri, ci)]
    err_nat = oracle.metrics.e_cw(nat, hi, lo, A[ri], B[:, ci])
    assert err < 1e-13
    if s == 16:
        assert err <= 2 * err_nat, (err, err_nat)


def test_large_zgemm_3m_sampled(ctx):
    n, s = 2048, 16
    A = synth.complex_phi_matrix(n, n, 1.0, synth.seed_for(4, n, 1.0, synth.ROLE_A),
                                 synth.seed_for(4, n, 1.0, synth.ROLE_A_IM))
    B = synth.complex_phi_matrix(n, n, 1.0, synth.seed_for(4, n, 1.0, synth.ROLE_B),
                                 synth.seed_for(4, n, 1.0, synth.ROLE_B_IM))
    C = host(ozk.ozk_zgemm_3m(ctx, s, dev(A), dev(B)))
    rng = np.random.default_rng(11)
    rows = rng.integers(0, n, 16)
    cols = rng.integers(0, n, 16)
    assert np.array_equal(C[rows, cols], s2.z3m_entries(A, B, s, rows, cols))


def fused(ctx, s, M, N, K, variant=ozk.OZK_S2_FUSED_CRT):
    ozk.ozk_config_set(ctx, ozk.OZK_OP_DGEMM, ozk.OZK_SCHEME2, s, M, N, K, (variant, 0, 4, 1))


@pytest.mark.parametrize("s", [1, 7, 12, 13, 16, 17, 20])
@pytest.mark.parametrize("shape", [(1, 1, 1), (63, 65, 127), (129, 200, 95), (70, 64, 0)])
def test_fused_crt_bit_exact(s, shape):
    """The GEMM with the CRT fused into it (no residue planes; 6, 8 or 10
    16-bit pieces per CRT sum by s) equals the oracle and the separate
    kernels, over several tiles with ragged edges and K = 0."""
    c = ozk.Context(0)
    try:
        M, N, K = shape
        A = synth.phi_matrix(M, K, 1.0, 1400 + s + M)
        B = synth.phi_matrix(K, N, 1.0, 1500 + s + N)
        fused(c, s, M, N, K)
        got = host(ozk.ozk_dgemm(c, ozk.OZK_SCHEME2, s, dev(A), dev(B), C=dev(np.full((M, N), np.nan))))
        # K = 0: the empty sum (beta = 0, so the NaNs of C are not read)
        assert np.array_equal(got, s2.s2_dgemm(A, B, s) if K else np.zeros((M, N)))
        fused(c, s, M, N, K, variant=3)
        assert np.array_equal(got, host(ozk.ozk_dgemm(c, ozk.OZK_SCHEME2, s, dev(A), dev(B))))
    finally:
        c.close()


def test_fused_crt_alpha_beta_edges():
    """Zero, tiny, huge, non-finite rows and columns, subnormal and overflowing
    products, alpha and beta: the fused epilogue rounds and scales like the
    separate CRT kernel."""
    s, M, N, K = 14, 70, 66, 50
    A = synth.phi_matrix(M, K, 1.0, 11)
    B = synth.phi_matrix(K, N, 1.0, 12)
    C0 = synth.phi_matrix(M, N, 1.0, 13)
    A[0] = 0
    A[1] *= 1e-300
    A[2] *= 1e300
    A[3, 4] = np.inf
    A[4] *= 1e-160
    A[65, :4] = [5e-324, -1e-310, 0.0, 2.0 ** -1060]
    B[:, 5] = 0
    B[7, 6] = np.nan
    B[:, 8] *= 1e-160
    B[:, 64] *= 1e10
    c = ozk.Context(0)
    try:
        fused(c, s, M, N, K)
        got = host(ozk.ozk_dgemm(c, ozk.OZK_SCHEME2, s, dev(A), dev(B), C=dev(C0), alpha=-1.5, beta=0.5))
        ref = s2.s2_dgemm(A, B, s, alpha=-1.5, beta=0.5, C=C0)
        assert np.array_equal(np.isnan(got), np.isnan(ref))
        ok = ~np.isnan(ref)
        assert np.array_equal(got[ok], ref[ok])
        got0 = host(ozk.ozk_dgemm(c, ozk.OZK_SCHEME2, s, dev(A), dev(B)))
        ref0 = s2.s2_dgemm(A, B, s)
        ok0 = ~np.isnan(ref0)
        assert np.array_equal(np.isnan(got0), np.isnan(ref0)) and np.array_equal(got0[ok0], ref0[ok0])
        assert 0 < abs(ref0[4, 8]) < np.finfo(np.float64).tiny and np.isinf(ref0[2, 64])
    finally:
        c.close()


def test_fused_crt_large_sampled():
    """8192 x 8192 x 2048 with s = 16, the shape where the residue planes are
    largest against the GEMM: sampled outputs against the oracle and the
    whole result against the separate kernels."""
    M, N, K, s = 8192, 8192, 2048, 16
    A = synth.phi_matrix(M, K, 1.0, synth.seed_for(3, M, 1.0, synth.ROLE_A))
    B = synth.phi_matrix(K, N, 1.0, synth.seed_for(3, N, 1.0, synth.ROLE_B))
    a, b = dev(A), dev(B)
    c = ozk.Context(0)
    try:
        fused(c, s, M, N, K)
        got = ozk.ozk_dgemm(c, ozk.OZK_SCHEME2, s, a, b)
        fused(c, s, M, N, K, variant=3)
        assert torch.equal(got, ozk.ozk_dgemm(c, ozk.OZK_SCHEME2, s, a, b))
        C = host(got)
        rng = np.random.default_rng(7)
        rows = np.concatenate([rng.integers(0, M, 30), [0, M - 1]])
        cols = np.concatenate([rng.integers(0, N, 30), [N - 1, 0]])
        assert np.array_equal(C[rows, cols], s2.s2_entries(A, B, s, rows, cols))
    finally:
        c.close()


# ------------------------------------------------ binary32 operands and results

@pytest.mark.parametrize("s", [1, 8, 11, 16, 20])
@pytest.mark.parametrize("shape", [(1, 1, 1), (63, 65, 127), (129, 130, 95)])
def test_sgemm_scheme2_bit_exact(ctx, s, shape):
    M, N, K = shape
    A = synth.phi_matrix(M, K, 1.0, 1600 + s + M).astype(np.float32)
    B = synth.phi_matrix(K, N, 1.0, 1700 + s + N).astype(np.float32)
    C = host(ozk.ozk_sgemm(ctx, ozk.OZK_SCHEME2, s, dev(A), dev(B)))
    assert C.dtype == np.float32 and np.array_equal(C, s2.s2_sgemm(A, B, s))


def test_sgemm_scheme2_edges_and_long_k():
    """Zero, tiny and huge rows, non-finite entries, binary32 underflow and
    overflow, alpha/beta; and K past the column-scale split (long-K path)."""
    s, M, N, K = 10, 40, 30, 50
    A = synth.phi_matrix(M, K, 1.0, 61).astype(np.float32)
    B = synth.phi_matrix(K, N, 1.0, 62).astype(np.float32)
    C0 = synth.phi_matrix(M, N, 1.0, 63).astype(np.float32)
    A[0] = 0
    A[1] *= np.float32(1e-38)
    A[2] *= np.float32(1e30)
    A[3, 4] = np.inf
    A[4] *= np.float32(1e-20)
    B[:, 5] = 0
    B[7, 6] = np.nan
    B[:, 8] *= np.float32(1e-20)
    B[:, 9] *= np.float32(1e20)
    c = ozk.Context(0)
    try:
        got = host(ozk.ozk_sgemm(c, ozk.OZK_SCHEME2, s, dev(A), dev(B), C=dev(C0), alpha=-1.5, beta=0.5))
        ref = s2.s2_sgemm(A, B, s, alpha=-1.5, beta=0.5, C=C0)
        assert np.array_equal(np.isnan(got), np.isnan(ref))
        ok = ~np.isnan(ref)
        assert np.array_equal(got[ok], ref[ok])
        ref0 = s2.s2_sgemm(A, B, s)
        got0 = host(ozk.ozk_sgemm(c, ozk.OZK_SCHEME2, s, dev(A), dev(B)))
        ok0 = ~np.isnan(ref0)
        assert np.array_equal(got0[ok0], ref0[ok0]) and np.isinf(ref0[2, 9]) and 0 < abs(ref0[4, 8]) < 1.2e-38
        # long K: the split column statistics
        A2 = synth.phi_matrix(20, 1100, 1.0, 64).astype(np.float32)
        B2 = synth.phi_matrix(1100, 300, 1.0, 65).astype(np.float32)
        assert np.array_equal(host(ozk.ozk_sgemm(c, ozk.OZK_SCHEME2, 9, dev(A2), dev(B2))), s2.s2_sgemm(A2, B2, 9))
    finally:
        c.close()


@pytest.mark.parametrize("s", [4, 9, 16])
@pytest.mark.parametrize("shape", [(1, 1, 1), (63, 65, 70), (130, 40, 96)])
def test_cgemm_3m_bit_exact(ctx, s, shape):
    M, N, K = shape
    A = synth.complex_phi_matrix(M, K, 1.0, 1800 + s, 1801 + s).astype(np.complex64)
    B = synth.complex_phi_matrix(K, N, 1.0, 1802 + s, 1803 + s).astype(np.complex64)
    C = host(ozk.ozk_cgemm_3m(ctx, s, dev(A), dev(B)))
    assert C.dtype == np.complex64 and np.array_equal(C, s2.z3m_cgemm(A, B, s))


def test_cgemm_3m_alpha_beta():
    s, M, N, K = 10, 30, 20, 40
    A = synth.complex_phi_matrix(M, K, 1.0, 1900, 1901).astype(np.complex64)
    B = synth.complex_phi_matrix(K, N, 1.0, 1902, 1903).astype(np.complex64)
    C0 = synth.complex_phi_matrix(M, N, 1.0, 1904, 1905).astype(np.complex64)
    al, be = 0.5 - 2j, -1 + 0.25j
    c = ozk.Context(0)
    try:
        got = host(ozk.ozk_cgemm_3m(c, s, dev(A), dev(B), C=dev(C0), alpha=al, beta=be))
        assert np.array_equal(got, s2.z3m_cgemm(A, B, s, alpha=al, beta=be, C=C0))
    finally:
        c.close()


@pytest.mark.parametrize("cplx", [False, True])
def test_row_pass_split_over_k(ctx, cplx):
    """Few long rows: the scales first, then the residues over (row block,
    K range) -- ragged K, padding rows and a non-finite row included."""
    M, N, K, s = 40, 30, 1500, 12
    if cplx:
        A = synth.complex_phi_matrix(M, K, 1.0, 2000, 2001)
        B = synth.complex_phi_matrix(K, N, 1.0, 2002, 2003)
    else:
        A = synth.phi_matrix(M, K, 1.0, 2000)
        B = synth.phi_matrix(K, N, 1.0, 2002)
    A[3, 1234] = np.nan
    A[5] = 0
    got = host(ozk.ozk_zgemm_3m(ctx, s, dev(A), dev(B)) if cplx else ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME2, s, dev(A), dev(B)))
    ref = s2.z3m_gemm(A, B, s) if cplx else s2.s2_dgemm(A, B, s)
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    ok = ~np.isnan(ref)
    assert np.array_equal(got[ok], ref[ok])
