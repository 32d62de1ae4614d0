"""Scheme I on the GPU against the CPU oracle, through the C ABI.

Bit-exact: exponents, packed slices (Eq. 1 and the interleaved layout of
Eq. 11), the raw INT32 diagonals of the fused kernel (Eq. 2) and the FP64
outputs (exact shift-reduce + one rounding, Eq. 3).  Sizes span several
workgroup tiles and ragged tails; large sizes are checked on sampled outputs
that the oracle computes one by one."""
import os

import numpy as np
import pytest

import oracle
import paper_2606_25453_amd as ozk
import synth

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


SHAPES = [(1, 1, 1), (63, 65, 127), (128, 128, 128), (129, 257, 95), (300, 200, 513), (64, 300, 33)]


@pytest.mark.parametrize("p", [1, 3, 4, 5, 8])
@pytest.mark.parametrize("shape", [(37, 70), (256, 128), (300, 513)])
def test_split_rows_bit_exact(ctx, p, shape):
    rows, K = shape
    X = synth.phi_matrix(rows, K, 2.0, 1000 + p)
    X[min(3, rows - 1)] = 0.0
    e, packed = ozk.ozk_s1_split_rows(ctx, p, dev(X))
    e = host(e)[:rows]
    assert np.array_equal(e, oracle.s1_row_exponents(X))
    D = host(ozk.unpack_s1(packed, rows, K, p))
    assert np.array_equal(D, oracle.s1_digits_a(X, e, p))
    # padding rows and padded k are zero
    full = host(ozk.unpack_s1(packed, ((rows + 255) // 256) * 256, ((K + 31) // 32) * 32, p))
    assert not full[:, rows:, :].any() and not full[:, :, K:].any()


@pytest.mark.parametrize("p", [3, 7])
@pytest.mark.parametrize("shape", [(5, 8190), (6, 9000), (3, 16384), (4, 16500)])
def test_split_rows_long_rows(ctx, p, shape):
    """Long rows (K around 8192 and 16384, ragged tails) with zero and tiny
    entries."""
    rows, K = shape
    X = synth.phi_matrix(rows, K, 2.0, 3000 + K)
    X[1] = 0.0
    X[2, : K // 2] *= 1e-200
    e, packed = ozk.ozk_s1_split_rows(ctx, p, dev(X))
    e = host(e)[:rows]
    assert np.array_equal(e, oracle.s1_row_exponents(X))
    D = host(ozk.unpack_s1(packed, rows, K, p))
    assert np.array_equal(D, oracle.s1_digits_a(X, e, p))


@pytest.mark.parametrize("p", [1, 2, 6, 8])
@pytest.mark.parametrize("shape", [(70, 37), (128, 256), (513, 300)])
def test_split_cols_bit_exact(ctx, p, shape):
    K, cols = shape
    X = synth.phi_matrix(K, cols, 2.0, 2000 + p)
    X[:, min(5, cols - 1)] = 0.0
    f, packed = ozk.ozk_s1_split_cols(ctx, p, dev(X))
    f = host(f)[:cols]
    assert np.array_equal(f, oracle.s1_col_exponents(X))
    D = host(ozk.unpack_s1(packed, cols, K, p))
    assert np.array_equal(D, oracle.s1_digits_b(X, f, p).transpose(0, 2, 1))


def test_interleaved_layout_matches_eq11(ctx):
    """Eq. 11 with t_K = 32: column block (c p + i) of the interleaved matrix
    holds slice i of K chunk c, so a row reads [A'_0 | A'_1 | A'_2 | A'_0 |
    ...] (the paper's p = 3 example); the blocks are stored one after the
    other, each as a contiguous 256-row slab."""
    p, rows, K = 3, 5, 96
    X = synth.phi_matrix(rows, K, 1.0, 3)
    e, packed = ozk.ozk_s1_split_rows(ctx, p, dev(X))
    blocks = host(packed)[: 256 * K * p].reshape(K * p // 32, 256, 32)
    Ahat = np.concatenate(list(blocks), axis=1)  # rows x pK, Eq. 11's matrix
    D = oracle.s1_digits_a(X, oracle.s1_row_exponents(X), p)
    for r in range(rows):
        for c in range(K // 32):
            for i in range(p):
                assert np.array_equal(Ahat[r, (c * p + i) * 32:(c * p + i + 1) * 32], D[i, r, c * 32:(c + 1) * 32])


@pytest.mark.parametrize("p", [1, 2, 4, 5, 7, 8])
@pytest.mark.parametrize("shape", [(63, 65, 127), (129, 257, 95), (256, 64, 320)])
def test_int32_diagonals_bit_exact(ctx, p, shape):
    M, N, K = shape
    A = synth.phi_matrix(M, K, 1.0, 3000 + p)
    B = synth.phi_matrix(K, N, 1.0, 3100 + p)
    e, pa = ozk.ozk_s1_split_rows(ctx, p, dev(A))
    f, pb = ozk.ozk_s1_split_cols(ctx, p, dev(B))
    Cd = host(ozk.ozk_s1_diagonals(ctx, p, M, N, K, pa, pb))
    D = oracle.s1_digits_a(A, oracle.s1_row_exponents(A), p).astype(np.int64)
    E = oracle.s1_digits_b(B, oracle.s1_col_exponents(B), p).astype(np.int64)
    for d in range(p):
        ref = sum(D[t] @ E[d - t] for t in range(d + 1))
        assert np.array_equal(Cd[d].astype(np.int64), ref), d


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("shape", SHAPES)
def test_dgemm_bit_exact(ctx, p, shape):
    M, N, K = shape
    A = synth.phi_matrix(M, K, 1.0, 4000 + 10 * p + M)
    B = synth.phi_matrix(K, N, 1.0, 4100 + 10 * p + N)
    C = host(ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME1, p, dev(A), dev(B)))
    assert np.array_equal(C, oracle.s1_dgemm(A, B, p))


@pytest.mark.parametrize("p", [2, 5, 7])
def test_dgemm_every_step_count(ctx, p):
    """K from 1 to 8 steps of 32, full and ragged: the software pipeline's
    prologue, the leading zero step of odd counts and the last pair."""
    M, N = 130, 70
    for steps in range(1, 9):
        for K in (32 * steps, 32 * steps - 5):
            A = synth.phi_matrix(M, K, 1.0, 5000 + K)
            B = synth.phi_matrix(K, N, 1.0, 5100 + K)
            C = host(ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME1, p, dev(A), dev(B)))
            assert np.array_equal(C, oracle.s1_dgemm(A, B, p)), (p, K)


def test_config1_uniform_128(ctx):
    """128^3, entries uniform in (-1, 1), p = 4: bit-exact, and compared with
    the naive and double-double references."""
    M = N = K = 128
    A = synth.uniform_matrix(M, K, synth.seed_for(1, M, 0.0, synth.ROLE_A))
    B = synth.uniform_matrix(K, N, synth.seed_for(1, M, 0.0, synth.ROLE_B))
    C = host(ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME1, 4, dev(A), dev(B)))
    assert np.array_equal(C, oracle.s1_dgemm(A, B, 4))
    hi, lo = oracle.gemm_dd(A, B)
    err = oracle.metrics.e_cw(C, hi, lo, A, B)
    assert 1e-12 < err < 1e-7  # p = 4 keeps 30 bits per operand


def test_alpha_beta_and_strides(ctx):
    M, N, K, p = 70, 90, 110, 6
    A = synth.phi_matrix(M, K, 1.0, 1)
    B = synth.phi_matrix(K, N, 1.0, 2)
    C0 = synth.phi_matrix(M, N, 1.0, 3)
    # strided views: leading dimensions larger than the row length
    Ab = dev(np.zeros((M, K + 7)))
    Ab[:, :K] = dev(A)
    Bb = dev(np.zeros((K, N + 3)))
    Bb[:, :N] = dev(B)
    Cb = dev(np.full((M, N + 5), np.nan))
    ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME1, p, Ab[:, :K], Bb[:, :N], C=Cb[:, :N], alpha=-2.5, beta=0.0)
    out = host(Cb)
    assert np.array_equal(out[:, :N], oracle.s1_dgemm(A, B, p, alpha=-2.5))
    assert np.isnan(out[:, N:]).all()  # untouched
    Cb[:, :N] = dev(C0)
    ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME1, p, Ab[:, :K], Bb[:, :N], C=Cb[:, :N], alpha=0.75, beta=-1.25)
    assert np.array_equal(host(Cb)[:, :N], oracle.s1_dgemm(A, B, p, alpha=0.75, beta=-1.25, C=C0))


def test_edge_values(ctx):
    M, N, K, p = 40, 33, 50, 8
    A = synth.phi_matrix(M, K, 1.0, 11)
    B = synth.phi_matrix(K, N, 1.0, 12)
    A[0] = 0.0
    B[:, 1] = 0.0
    A[2] *= 1e-300
    A[3] *= 1e300
    A[4, :5] = [5e-324, -2.0 ** -1074, 1e-310, 0.0, -3e-320]
    A[5, 7] = np.nan
    B[9, 4] = -np.inf
    A[6] = A[7] = 1e-200  # products underflow into subnormals
    B[:, 8] *= 1e-150
    C = host(ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME1, p, dev(A), dev(B)))
    ref = oracle.s1_dgemm(A, B, p)
    assert np.array_equal(np.isnan(C), np.isnan(ref))
    ok = ~np.isnan(ref)
    assert np.array_equal(C[ok], ref[ok])
    assert np.isnan(C[5]).all() and np.isnan(C[:, 4]).all()


def test_empty_dimensions(ctx):
    for (M, N, K) in [(0, 5, 7), (5, 0, 7), (5, 7, 0), (0, 0, 0)]:
        A = dev(np.ones((M, K)))
        B = dev(np.ones((K, N)))
        C = dev(np.full((M, N), 7.0))
        ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME1, 3, A, B, C=C, alpha=1.0, beta=0.0)
        assert np.array_equal(host(C), np.zeros((M, N)))


def test_k_runs_fold_exactly():
    """Shorter overflow-free K runs (forced through ozk_set_k_split) fold into
    the same result as one run."""
    c2 = ozk.Context(0)
    for bad in (-32, 1, 31, 33):
        with pytest.raises(ozk.OzkError):
            ozk.ozk_set_k_split(c2, bad)
    ozk.ozk_set_k_split(c2, 64)
    M, N, K, p = 150, 70, 333, 8
    A = synth.phi_matrix(M, K, 1.0, 21)
    B = synth.phi_matrix(K, N, 1.0, 22)
    C = host(ozk.ozk_dgemm(c2, ozk.OZK_SCHEME1, p, dev(A), dev(B)))
    assert np.array_equal(C, oracle.s1_dgemm(A, B, p))
    c2.close()


def test_invalid_arguments(ctx):
    A = dev(np.ones((4, 4)))
    with pytest.raises(ozk.OzkError) as ei:
        ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME1, 9, A, A)
    assert ei.value.status == ozk.OZK_ERR_UNSUPPORTED
    with pytest.raises(ozk.OzkError) as ei:
        ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME1, 0, A, A)
    assert ei.value.status == ozk.OZK_ERR_UNSUPPORTED
    small = torch.empty(16, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(ozk.OzkError) as ei:
        ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME1, 4, A, A, ws=small)
    assert ei.value.status == ozk.OZK_ERR_WORKSPACE
    lib = ozk.library()
    st = lib.ozk_dgemm(ctx.handle, 1, 4, 4, 4, 4, 1.0, A.data_ptr(), 3, A.data_ptr(), 4, 0.0, A.data_ptr(), 4,
                       None, 0, None)
    assert st == ozk.OZK_ERR_INVALID_ARG and lib.ozk_last_arg(ctx.handle) == 9  # lda < K


def test_deterministic(ctx):
    A = synth.phi_matrix(200, 300, 2.0, 31)
    B = synth.phi_matrix(300, 150, 2.0, 32)
    a, b = dev(A), dev(B)
    r1 = host(ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME1, 7, a, b))
    r2 = host(ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME1, 7, a, b))
    assert np.array_equal(r1, r2)


@pytest.mark.parametrize("n,p", [(2048, 8), (8192, 8), (8192, 7)])
def test_large_sampled_bit_exact(ctx, n, p):
    """Full-size problems: sampled outputs against the oracle computed entry
    by entry, plus accuracy against double-double on a sampled block."""
    A = synth.phi_matrix(n, n, 1.0, synth.seed_for(2, n, 1.0, synth.ROLE_A))
    B = synth.phi_matrix(n, n, 1.0, synth.seed_for(2, n, 1.0, synth.ROLE_B))
    a, b = dev(A), dev(B)
    C = host(ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME1, p, a, b))
    rng = np.random.default_rng(n + p)
    rows = np.concatenate([rng.integers(0, n, 200), [0, n - 1, n - 1, 0]])
    cols = np.concatenate([rng.integers(0, n, 200), [0, n - 1, 0, n - 1]])
    ref = oracle.s1_entries(A, B, p, rows, cols)
    assert np.array_equal(C[rows, cols], ref)
    ri = rng.choice(n, 8, replace=False)
    ci = rng.choice(n, 8, replace=False)
    hi, lo = oracle.gemm_dd(A[ri], B[:, ci])
    sub = C[np.ix_(ri, ci)]
    err = oracle.metrics.e_cw(sub, hi, lo, A[ri], B[:, ci])
    nat = host(torch.matmul(a, b))[np.ix_(ri, ci)]
    err_nat = oracle.metrics.e_cw(nat, hi, lo, A[ri], B[:, ci])
    assert err < 1e-13
    if p == 8:
        assert err <= 2 * err_nat, (err, err_nat)


# ------------------------------------------------ binary32 operands and result

def f32(x):
    return np.ascontiguousarray(x, np.float32)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 6, 8])
@pytest.mark.parametrize("shape", SHAPES)
def test_sgemm_bit_exact(ctx, p, shape):
    """ozk_sgemm (binary32 in and out) equals the oracle bit for bit over
    several tiles with ragged edges."""
    M, N, K = shape
    A = f32(synth.phi_matrix(M, K, 1.0, 6000 + 10 * p + M))
    B = f32(synth.phi_matrix(K, N, 1.0, 6100 + 10 * p + N))
    C = host(ozk.ozk_sgemm(ctx, ozk.OZK_SCHEME1, p, dev(A), dev(B), C=dev(np.full((M, N), np.nan, np.float32))))
    assert C.dtype == np.float32 and np.array_equal(C, oracle.s1_sgemm(A, B, p))


def test_sgemm_edges_alpha_beta_and_empty(ctx):
    """Zero, tiny (binary32 subnormal) and huge rows, products that underflow
    to binary32 subnormals or overflow to infinity, non-finite entries,
    alpha/beta, and K = 0."""
    p, M, N, K = 4, 70, 66, 50
    A = f32(synth.phi_matrix(M, K, 1.0, 31))
    B = f32(synth.phi_matrix(K, N, 1.0, 32))
    C0 = f32(synth.phi_matrix(M, N, 1.0, 33))
    A[0] = 0
    A[1] *= np.float32(1e-38)
    A[2] *= np.float32(1e30)
    A[3, 4] = np.inf
    A[4, :3] = [1e-45, -3e-44, 0.0]
    A[65] *= np.float32(1e-20)
    B[:, 5] = 0
    B[7, 6] = np.nan
    B[:, 8] *= np.float32(1e-20)
    B[:, 64] *= np.float32(1e20)
    got = host(ozk.ozk_sgemm(ctx, ozk.OZK_SCHEME1, p, dev(A), dev(B), C=dev(C0), alpha=-1.5, beta=0.5))
    ref = oracle.s1_sgemm(A, B, p, alpha=-1.5, beta=0.5, C=C0)
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    ok = ~np.isnan(ref)
    assert np.array_equal(got[ok], ref[ok])
    got0 = host(ozk.ozk_sgemm(ctx, ozk.OZK_SCHEME1, p, dev(A), dev(B)))
    ref0 = oracle.s1_sgemm(A, B, p)
    ok0 = ~np.isnan(ref0)
    assert np.array_equal(np.isnan(got0), np.isnan(ref0)) and np.array_equal(got0[ok0], ref0[ok0])
    assert 0 < abs(ref0[65, 8]) < np.finfo(np.float32).tiny and np.isinf(ref0[2, 64])
    C = dev(np.full((5, 3), 7.0, np.float32))
    ozk.ozk_sgemm(ctx, ozk.OZK_SCHEME1, p, dev(np.ones((5, 0), np.float32)), dev(np.ones((0, 3), np.float32)), C=C)
    assert np.array_equal(host(C), np.zeros((5, 3), np.float32))
    one = dev(np.ones((4, 4), np.float32))
    big = torch.empty(1 << 20, dtype=torch.uint8, device="cuda:0")
    for bad in (0, 9):
        with pytest.raises(ozk.OzkError) as ei:
            ozk.ozk_sgemm(ctx, ozk.OZK_SCHEME1, bad, one, one, ws=big)
        assert ei.value.status == ozk.OZK_ERR_UNSUPPORTED
    with pytest.raises(ozk.OzkError) as ei:
        ozk.ozk_sgemm(ctx, ozk.OZK_SCHEME1, p, one, one, ws=torch.empty(1, dtype=torch.uint8, device="cuda:0"))
    assert ei.value.status == ozk.OZK_ERR_WORKSPACE


def test_sgemm_k_runs_and_configs(ctx):
    """The K split (128-bit partials folded exactly, then the binary32
    rounding) and every tile variant give the same binary32 result."""
    p, M, N, K = 3, 130, 70, 700
    A = f32(synth.phi_matrix(M, K, 1.0, 41))
    B = f32(synth.phi_matrix(K, N, 1.0, 42))
    ref = oracle.s1_sgemm(A, B, p)
    c = ozk.Context(0)
    try:
        for cfg in [(0, 0, 4, 1), (1, 1, 2, 3), (2, 0, 8, 5), (3, 1, 1, 2)]:
            ozk.ozk_config_set(c, ozk.OZK_OP_DGEMM, ozk.OZK_SCHEME1, p, M, N, K, cfg)
            assert np.array_equal(host(ozk.ozk_sgemm(c, ozk.OZK_SCHEME1, p, dev(A), dev(B))), ref), cfg
    finally:
        c.close()


def test_sgemm_1024_against_oracle_and_native_error(ctx):
    """1024 x 1024 x 512 at p = 4: bit-exact against the oracle, and the error
    against the double-double reference at the level of native binary32
    (p = 3 leaves about 2^-16: the slices carry 8p - 2 bits relative to the
    row's largest entry)."""
    p, M, N, K = 4, 1024, 1024, 512
    A = f32(synth.phi_matrix(M, K, 1.0, 51))
    B = f32(synth.phi_matrix(K, N, 1.0, 52))
    a, b = dev(A), dev(B)
    C = host(ozk.ozk_sgemm(ctx, ozk.OZK_SCHEME1, p, a, b))
    assert np.array_equal(C, oracle.s1_sgemm(A, B, p))
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    ri, ci = np.arange(0, M, 97), np.arange(0, N, 89)
    hi, lo = oracle.gemm_dd(A64[ri], B64[:, ci])
    err = oracle.metrics.e_cw(C[np.ix_(ri, ci)].astype(np.float64), hi, lo, A64[ri], B64[:, ci])
    nat = host(torch.matmul(a, b))[np.ix_(ri, ci)].astype(np.float64)
    err_nat = oracle.metrics.e_cw(nat, hi, lo, A64[ri], B64[:, ci])
    assert err < 4 * max(err_nat, 2.0 ** -24), (err, err_nat)


# ------------------------------------------------ unfused baseline (ablation)

@pytest.mark.parametrize("p", [1, 3, 7, 8])
@pytest.mark.parametrize("shape", [(1, 1, 1), (129, 257, 95), (300, 200, 513), (70, 40, 0)])
def test_unfused_baseline_equals_fused(ctx, p, shape):
    """One GEMM per slice pair with INT32 planes through HBM, then the
    reconstruction: the same result as the fused kernel and the oracle."""
    M, N, K = shape
    A = synth.phi_matrix(M, K, 1.0, 7000 + p + M)
    B = synth.phi_matrix(K, N, 1.0, 7100 + p + N)
    C0 = synth.phi_matrix(M, N, 1.0, 7200 + p)
    got = host(ozk.ozk_s1_dgemm_unfused(ctx, p, dev(A), dev(B), C=dev(C0), alpha=0.75, beta=-2.0))
    fused = host(ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME1, p, dev(A), dev(B), C=dev(C0), alpha=0.75, beta=-2.0))
    assert np.array_equal(got, fused)
    if K:
        assert np.array_equal(got, oracle.s1_dgemm(A, B, p, alpha=0.75, beta=-2.0, C=C0))


def test_unfused_baseline_k_limit(ctx):
    """K = 131071 is the longest single INT32 plane per pair; beyond it the
    baseline refuses (the fused path splits K instead)."""
    A = synth.phi_matrix(2, 131071, 1.0, 7300)
    B = synth.phi_matrix(131071, 3, 1.0, 7301)
    got = host(ozk.ozk_s1_dgemm_unfused(ctx, 2, dev(A), dev(B)))
    assert np.array_equal(got, host(ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME1, 2, dev(A), dev(B))))
    A2, B2 = dev(np.ones((2, 131072))), dev(np.ones((131072, 3)))
    with pytest.raises(ozk.OzkError) as ei:
        ozk.ozk_s1_dgemm_unfused(ctx, 2, A2, B2, ws=torch.empty(1 << 24, dtype=torch.uint8, device="cuda:0"))
    assert ei.value.status == ozk.OZK_ERR_UNSUPPORTED
