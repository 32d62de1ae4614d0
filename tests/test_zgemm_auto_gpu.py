"""The automatic ZGEMM (ozk_zgemm_auto): the modulus count decided on the
device equals the oracle's complex Scheme II bound, the result is
bit-identical to ozk_zgemm_3m at that count and to the oracle, it meets the
tolerance whenever the count is proven, and the call can be replayed from a
graph."""
import numpy as np
import pytest

import oracle
import paper_2606_25453_amd as ozk
import synth
from oracle import scheme2 as s2
from oracle import selector as sel

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


@pytest.mark.parametrize("M,K,N,phi", [(33, 70, 41, 1.0), (130, 257, 65, 2.5), (1, 5, 2, 0.0)])
def test_zgemm_auto_decision_and_result(ctx, M, K, N, phi):
    A = synth.complex_phi_matrix(M, K, phi, 4000 + M, 4001 + M)
    B = synth.complex_phi_matrix(K, N, phi, 4002 + M, 4003 + M)
    C0 = synth.complex_phi_matrix(M, N, 1.0, 4004, 4005)
    dA, dB = dev(A), dev(B)
    hi, lo = oracle.zgemm_dd(A, B)
    for tol in (1e-5, 1e-9, 1e-13, 1e-16):
        C, info = ozk.ozk_zgemm_auto(ctx, tol, dA, dB, C=dev(C0), alpha=0.5 - 1j, beta=2 + 0.25j)
        info = host(info)
        sb = sel.s_bound_complex(A, B, tol)
        assert info[4] == 2 and info[6] == sb and info[5] == min(sb, 20), (tol, info.tolist(), sb)
        s = int(info[5])
        got = host(C)
        assert np.array_equal(got, host(ozk.ozk_zgemm_3m(ctx, s, dA, dB, C=dev(C0), alpha=0.5 - 1j, beta=2 + 0.25j)))
        if M * N * K <= 200000:
            assert np.array_equal(got, s2.z3m_gemm(A, B, s, alpha=0.5 - 1j, beta=2 + 0.25j, C=C0))
        if sb <= 20:
            plain = host(ozk.ozk_zgemm_auto(ctx, tol, dA, dB)[0])
            assert oracle.metrics.e_cw(plain, hi, lo, A, B) <= tol
    f = ozk.ozk_get_flags(ctx)
    assert f & ozk.OZK_FLAG_SELECTOR_FALLBACK and f & ozk.OZK_FLAG_SCHEME2_CHOSEN
    assert bool(f & ozk.OZK_FLAG_S_UNPROVEN) == (sel.s_bound_complex(A, B, 1e-16) > 20)


def test_zgemm_auto_graph_replay(ctx):
    M, K, N = 150, 200, 90
    A = dev(synth.complex_phi_matrix(M, K, 1.5, 4100, 4101))
    B = dev(synth.complex_phi_matrix(K, N, 1.5, 4102, 4103))
    C = torch.zeros((M, N), dtype=torch.complex128, device="cuda:0")
    ws = torch.empty(ozk.ozk_workspace_size(ctx, ozk.OZK_OP_ZGEMM, ozk.OZK_SCHEME2, M, N, K, 0), dtype=torch.uint8,
                     device="cuda:0")
    info = torch.zeros(ozk.OZK_SELECTOR_INFO, dtype=torch.int32, device="cuda:0")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        ozk.ozk_zgemm_auto(ctx, 1e-12, A, B, C=C, ws=ws, info=info, stream=side)
        torch.cuda.synchronize()
        eager = host(C).copy()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            ozk.ozk_zgemm_auto(ctx, 1e-12, A, B, C=C, ws=ws, info=info, stream=side)
    torch.cuda.current_stream().wait_stream(side)
    for rep in range(3):
        C.fill_(complex(rep, 1.0))
        info.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(C), eager), rep
        assert host(info)[4] == 2


def test_zgemm_auto_nonfinite_and_errors(ctx):
    A = synth.complex_phi_matrix(20, 30, 1.0, 4200, 4201)
    B = synth.complex_phi_matrix(30, 10, 1.0, 4202, 4203)
    A[3, 4] = complex(np.nan, 1.0)
    C, info = ozk.ozk_zgemm_auto(ctx, 1e-10, dev(A), dev(B))
    got = host(C)
    assert np.isnan(got[3].real).all() and np.isfinite(np.delete(got, 3, axis=0).real).all()
    assert ozk.ozk_get_flags(ctx) & ozk.OZK_FLAG_NONFINITE
    for tol in (0.0, 1.0, float("nan")):
        with pytest.raises(ozk.OzkError) as ei:
            ozk.ozk_zgemm_auto(ctx, tol, dev(A), dev(B))
        assert ei.value.status == ozk.OZK_ERR_INVALID_ARG and ei.value.arg == 2
