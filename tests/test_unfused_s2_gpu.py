"""The unfused Scheme II and 3M baselines (INT32 planes through HBM, the
paper's naive forms) are bit-identical to the fused calls and to the
oracle."""
import numpy as np
import pytest

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


@pytest.mark.parametrize("s", [1, 8, 14, 20])
@pytest.mark.parametrize("shape", [(64, 64, 64), (200, 131, 97)])
def test_unfused_scheme2_real(ctx, s, shape):
    M, N, K = shape
    A = synth.phi_matrix(M, K, 1.0, 3600 + s)
    B = synth.phi_matrix(K, N, 1.0, 3601 + s)
    C0 = synth.phi_matrix(M, N, 1.0, 3602)
    got = host(ozk.ozk_s2_gemm_unfused(ctx, s, dev(A), dev(B), C=dev(C0), alpha=0.75, beta=-2.0))
    assert np.array_equal(got, s2.s2_dgemm(A, B, s, alpha=0.75, beta=-2.0, C=C0))
    fused = host(ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME2, s, dev(A), dev(B), C=dev(C0), alpha=0.75, beta=-2.0))
    assert np.array_equal(got, fused)


@pytest.mark.parametrize("s", [1, 12, 16])
@pytest.mark.parametrize("shape", [(64, 64, 64), (150, 99, 75)])
def test_unfused_3m(ctx, s, shape):
    M, N, K = shape
    A = synth.complex_phi_matrix(M, K, 1.0, 3700 + s, 3701 + s)
    B = synth.complex_phi_matrix(K, N, 1.0, 3702 + s, 3703 + s)
    got = host(ozk.ozk_s2_gemm_unfused(ctx, s, dev(A), dev(B), alpha=1 - 1j))
    assert np.array_equal(got, s2.z3m_gemm(A, B, s, alpha=1 - 1j))
    assert np.array_equal(got, host(ozk.ozk_zgemm_3m(ctx, s, dev(A), dev(B), alpha=1 - 1j)))


def test_unfused_scheme2_limits(ctx):
    A = dev(np.ones((4, 131072)))
    B = dev(np.ones((131072, 4)))
    with pytest.raises(ozk.OzkError) as ei:
        ozk.ozk_s2_gemm_unfused(ctx, 8, A, B)
    assert ei.value.status == ozk.OZK_ERR_UNSUPPORTED and ei.value.arg == 6
    K = 131071  # the longest K whose INT32 planes stay exact: all residues at their extreme
    A = dev(np.full((2, K), -1.0))
    B = dev(np.full((K, 3), 1.0))
    got = host(ozk.ozk_s2_gemm_unfused(ctx, 20, A, B))
    assert np.array_equal(got, host(ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME2, 20, A, B)))
    assert np.array_equal(got, np.full((2, 3), -float(K)))


@pytest.mark.parametrize("cplx,s", [(False, 14), (True, 16)])
def test_unfused_at_the_measured_size(ctx, cplx, s):
    """4096^3, the size the ablation is measured at: the unfused result is the
    fused one everywhere and the oracle's on sampled rows and columns."""
    n = 4096
    if cplx:
        A = torch.complex(synth.phi_matrix_device(n, n, 1.0, 5300), synth.phi_matrix_device(n, n, 1.0, 5302))
        B = torch.complex(synth.phi_matrix_device(n, n, 1.0, 5301), synth.phi_matrix_device(n, n, 1.0, 5303))
        fused = ozk.ozk_zgemm_3m(ctx, s, A, B)
    else:
        A = synth.phi_matrix_device(n, n, 1.0, 5300)
        B = synth.phi_matrix_device(n, n, 1.0, 5301)
        fused = ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME2, s, A, B)
    got = ozk.ozk_s2_gemm_unfused(ctx, s, A, B)
    torch.cuda.synchronize()
    assert torch.equal(got, fused)
    rng = np.random.default_rng(s)
    rows = np.unique(rng.integers(0, n, 10))
    cols = np.unique(rng.integers(0, n, 10))
    r, c = torch.from_numpy(rows).cuda(), torch.from_numpy(cols).cuda()
    As, Bs = A.index_select(0, r).cpu().numpy(), B.index_select(1, c).cpu().numpy()
    sub = got.index_select(0, r).index_select(1, c).cpu().numpy()
    assert np.array_equal(sub, s2.z3m_gemm(As, Bs, s) if cplx else s2.s2_dgemm(As, Bs, s))
