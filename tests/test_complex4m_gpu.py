"""Scheme I complex GEMM by 4M (ozk_zgemm / ozk_cgemm with OZK_SCHEME1) on the
GPU against the CPU oracle, bit for bit, through the C ABI: the real
embedding's slices and exponents, the Scheme I product of the embedded
matrices (exact integer parts, one rounding each) and the complex update."""
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


def same(got, ref):
    """Bit-equal, NaN where the reference is NaN (real and imaginary parts)."""
    for part in (np.real, np.imag):
        g, r = part(got), part(ref)
        assert np.array_equal(np.isnan(g), np.isnan(r))
        ok = ~np.isnan(r)
        assert np.array_equal(g[ok], r[ok])


@pytest.mark.parametrize("p", [1, 3, 4, 6, 7, 8])
@pytest.mark.parametrize("shape", [(64, 64, 64), (131, 97, 75), (300, 257, 130)])
def test_zgemm_4m_bit_exact(ctx, p, shape):
    M, N, K = shape
    A = synth.complex_phi_matrix(M, K, 1.0, 3000 + p, 3001 + p)
    B = synth.complex_phi_matrix(K, N, 1.0, 3002 + p, 3003 + p)
    got = host(ozk.ozk_zgemm(ctx, ozk.OZK_SCHEME1, p, dev(A), dev(B)))
    assert np.array_equal(got, oracle.s1_zgemm(A, B, p))


def test_zgemm_4m_alpha_beta_strides_and_edges(ctx):
    M, N, K, p = 70, 45, 90, 7
    A = synth.complex_phi_matrix(M, K, 2.0, 3100, 3101)
    B = synth.complex_phi_matrix(K, N, 2.0, 3102, 3103)
    A[0] = 0
    A[1] = A[1].real  # a real row
    A[2] *= 1e-300
    A[3, 4] = complex(np.nan, 0.0)
    B[:, 5] = 1j * B[:, 5].imag  # an imaginary column
    B[7, 6] = complex(0.0, np.inf)
    B[:, 8] *= 1e250
    C0 = synth.complex_phi_matrix(M, N, 1.0, 3104, 3105)
    al, be = 0.5 - 2j, -1 + 0.25j
    got = host(ozk.ozk_zgemm(ctx, ozk.OZK_SCHEME1, p, dev(A), dev(B), C=dev(C0), alpha=al, beta=be))
    same(got, oracle.s1_zgemm(A, B, p, alpha=al, beta=be, C=C0))
    assert np.isnan(got[3].real).all() and np.isnan(got[:, 6].imag).all()
    # beta = 0: C is not read (NaN there does not leak)
    got0 = host(ozk.ozk_zgemm(ctx, ozk.OZK_SCHEME1, p, dev(A), dev(B), C=dev(np.full((M, N), np.nan + 0j))))
    same(got0, oracle.s1_zgemm(A, B, p))
    # row-major views with leading dimensions larger than the width
    Abig = synth.complex_phi_matrix(M, K + 9, 1.0, 3106, 3107)
    Bbig = synth.complex_phi_matrix(K, N + 5, 1.0, 3108, 3109)
    Cbig = dev(np.zeros((M, N + 3), np.complex128))
    ozk.ozk_zgemm(ctx, ozk.OZK_SCHEME1, p, dev(Abig)[:, :K], dev(Bbig)[:, :N], C=Cbig[:, :N])
    assert np.array_equal(host(Cbig)[:, :N], oracle.s1_zgemm(Abig[:, :K], Bbig[:, :N], p))


def test_zgemm_4m_k_runs_fold_exactly():
    """K runs of 64 of the embedded 2K (the exact 128-bit fold)."""
    c2 = ozk.Context(0)
    ozk.ozk_set_k_split(c2, 64)
    M, N, K, p = 90, 60, 170, 8
    A = synth.complex_phi_matrix(M, K, 1.0, 3200, 3201)
    B = synth.complex_phi_matrix(K, N, 1.0, 3202, 3203)
    assert np.array_equal(host(ozk.ozk_zgemm(c2, ozk.OZK_SCHEME1, p, dev(A), dev(B))), oracle.s1_zgemm(A, B, p))
    c2.close()


def test_zgemm_scheme2_is_3m(ctx):
    M, N, K, s = 77, 66, 55, 14
    A = synth.complex_phi_matrix(M, K, 1.0, 3300, 3301)
    B = synth.complex_phi_matrix(K, N, 1.0, 3302, 3303)
    got = host(ozk.ozk_zgemm(ctx, ozk.OZK_SCHEME2, s, dev(A), dev(B), alpha=2 - 1j))
    assert np.array_equal(got, s2.z3m_gemm(A, B, s, alpha=2 - 1j))


def test_zgemm_empty_and_invalid(ctx):
    for (M, N, K) in [(0, 4, 3), (4, 0, 3), (4, 3, 0)]:
        C = dev(np.full((M, N), 5.0 + 1j))
        ozk.ozk_zgemm(ctx, ozk.OZK_SCHEME1, 4, dev(np.ones((M, K), np.complex128)),
                      dev(np.ones((K, N), np.complex128)), C=C)
        assert np.array_equal(host(C), np.zeros((M, N), np.complex128))
    A = dev(np.ones((4, 4), np.complex128))
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda:0")
    for bad in (0, 9):
        with pytest.raises(ozk.OzkError) as ei:
            ozk.ozk_zgemm(ctx, ozk.OZK_SCHEME1, bad, A, A, ws=ws)
        assert ei.value.status == ozk.OZK_ERR_UNSUPPORTED and ei.value.arg == 3
    small = torch.empty(16, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(ozk.OzkError) as ei:
        ozk.ozk_zgemm(ctx, ozk.OZK_SCHEME1, 4, A, A, ws=small)
    assert ei.value.status == ozk.OZK_ERR_WORKSPACE and ei.value.arg == 15


@pytest.mark.parametrize("p", [2, 4])
@pytest.mark.parametrize("shape", [(64, 64, 64), (150, 99, 140)])
def test_cgemm_4m_bit_exact(ctx, p, shape):
    M, N, K = shape
    A = synth.complex_phi_matrix(M, K, 1.0, 3400 + p, 3401 + p).astype(np.complex64)
    B = synth.complex_phi_matrix(K, N, 1.0, 3402 + p, 3403 + p).astype(np.complex64)
    C0 = synth.complex_phi_matrix(M, N, 1.0, 3404, 3405).astype(np.complex64)
    got = host(ozk.ozk_cgemm(ctx, ozk.OZK_SCHEME1, p, dev(A), dev(B), C=dev(C0), alpha=1.5 + 0.5j, beta=-0.25j))
    assert np.array_equal(got, oracle.s1_cgemm(A, B, p, alpha=1.5 + 0.5j, beta=-0.25j, C=C0))
    got2 = host(ozk.ozk_cgemm(ctx, ozk.OZK_SCHEME2, 8, dev(A), dev(B)))
    assert np.array_equal(got2, s2.z3m_cgemm(A, B, 8))


@pytest.mark.parametrize("n,p", [(2048, 7), (4096, 7), (8192, 7)])
def test_zgemm_4m_large_sampled(ctx, n, p):
    """Full-size 4M ZGEMM: sampled rows and columns against the oracle (the
    exponents of a row of A and a column of B depend on nothing else), and
    E_cw against double-double within the 1e-13 gate."""
    from oracle import metrics
    A = torch.complex(synth.phi_matrix_device(n, n, 1.0, 3500), synth.phi_matrix_device(n, n, 1.0, 3502))
    B = torch.complex(synth.phi_matrix_device(n, n, 1.0, 3501), synth.phi_matrix_device(n, n, 1.0, 3503))
    C = ozk.ozk_zgemm(ctx, ozk.OZK_SCHEME1, p, A, B)
    rng = np.random.default_rng(n)
    rows = np.unique(np.concatenate([rng.integers(0, n, 14), [0, n - 1]]))
    cols = np.unique(np.concatenate([rng.integers(0, n, 14), [0, n - 1]]))
    r, c = torch.from_numpy(rows).cuda(), torch.from_numpy(cols).cuda()
    As, Bs = A.index_select(0, r).cpu().numpy(), B.index_select(1, c).cpu().numpy()
    got = host(C.index_select(0, r).index_select(1, c))
    assert np.array_equal(got, oracle.s1_zgemm(As, Bs, p))
    hi, lo = oracle.zgemm_dd(As, Bs)
    assert metrics.e_cw(got, hi, lo, As, Bs) <= 1e-13
