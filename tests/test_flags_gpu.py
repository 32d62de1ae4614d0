"""The asynchronous condition flags (ozk_get_flags): raised by non-finite
inputs in every whole call, by the automatic path's decisions, taken and
cleared atomically."""
import numpy as np
import pytest

import paper_2606_25453_amd as ozk
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture()
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = ozk.Context(0)
    yield c
    c.close()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def test_clean_calls_raise_nothing(ctx):
    A = dev(synth.phi_matrix(50, 40, 1.0, 1))
    B = dev(synth.phi_matrix(40, 30, 1.0, 2))
    ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME1, 7, A, B)
    ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME2, 12, A, B)
    assert ozk.ozk_get_flags(ctx) == 0


@pytest.mark.parametrize("where", ["a_row", "b_col"])
def test_nonfinite_input_in_every_call(ctx, where):
    M, N, K = 40, 30, 50
    A = synth.phi_matrix(M, K, 1.0, 3)
    B = synth.phi_matrix(K, N, 1.0, 4)
    Z = synth.complex_phi_matrix(M, K, 1.0, 5, 6)
    W = synth.complex_phi_matrix(K, N, 1.0, 7, 8)
    if where == "a_row":
        A[3, 7] = np.nan
        Z[3, 7] = complex(1.0, np.inf)
    else:
        B[9, 4] = -np.inf
        W[9, 4] = complex(np.nan, 0.0)
    a, b, z, w = dev(A), dev(B), dev(Z), dev(W)
    calls = [
        lambda: ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME1, 5, a, b),
        lambda: ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME2, 9, a, b),
        lambda: ozk.ozk_dgemm_t(ctx, ozk.OZK_SCHEME1, 5, a.T.contiguous(), b, trans_a=True),
        lambda: ozk.ozk_dgemm_noalloc(ctx, ozk.OZK_SCHEME1, 5, a, b),
        lambda: ozk.ozk_sgemm(ctx, ozk.OZK_SCHEME1, 3, a.float(), b.float()),
        lambda: ozk.ozk_sgemm(ctx, ozk.OZK_SCHEME2, 8, a.float(), b.float()),
        lambda: ozk.ozk_s1_dgemm_unfused(ctx, 4, a, b),
        lambda: ozk.ozk_s2_gemm_unfused(ctx, 8, a, b),
        lambda: ozk.ozk_zgemm_3m(ctx, 10, z, w),
        lambda: ozk.ozk_zgemm(ctx, ozk.OZK_SCHEME1, 6, z, w),
        lambda: ozk.ozk_cgemm(ctx, ozk.OZK_SCHEME1, 3, z.to(torch.complex64), w.to(torch.complex64)),
        lambda: ozk.ozk_cgemm_3m(ctx, 8, z.to(torch.complex64), w.to(torch.complex64)),
    ]
    for i, call in enumerate(calls):
        call()
        assert ozk.ozk_get_flags(ctx) == ozk.OZK_FLAG_NONFINITE, i
        assert ozk.ozk_get_flags(ctx) == 0, i  # taken and cleared


def test_batch_raises_the_nonfinite_flag(ctx):
    probs = []
    for i, (M, N, K) in enumerate([(40, 30, 20), (17, 70, 33)]):
        A = synth.phi_matrix(M, K, 1.0, 20 + i)
        B = synth.phi_matrix(K, N, 1.0, 30 + i)
        if i == 1:
            B[2, 5] = np.nan
        probs.append((dev(A), dev(B), torch.zeros((M, N), dtype=torch.float64, device="cuda:0")))
    plan = ozk.BatchPlan(ctx, ozk.OZK_OP_DGEMM, ozk.OZK_SCHEME2, 10, probs)
    plan.run()
    assert ozk.ozk_get_flags(ctx) == ozk.OZK_FLAG_NONFINITE
    probs[1][1][2, 5] = 1.0
    plan.run()
    assert ozk.ozk_get_flags(ctx) == 0


def test_auto_path_decision_flags(ctx):
    A = dev(synth.phi_matrix(64, 64, 1.0, 40))
    B = dev(synth.phi_matrix(64, 64, 1.0, 41))
    # no network loaded: the bound decides
    ozk.ozk_dgemm_auto(ctx, 1e-10, A, B)
    f = ozk.ozk_get_flags(ctx)
    assert f & ozk.OZK_FLAG_SELECTOR_FALLBACK and not f & ozk.OZK_FLAG_NONFINITE
    # entries spanning more exponents than 8 slices carry: Scheme II
    X = synth.phi_matrix(64, 64, 1.0, 42)
    X[:, 0] *= 2.0 ** 200
    info = torch.zeros(ozk.OZK_SELECTOR_INFO, dtype=torch.int32, device="cuda:0")
    ozk.ozk_dgemm_auto(ctx, 1e-14, dev(X), B, info=info)
    f = ozk.ozk_get_flags(ctx)
    if int(info[4]) == 2:
        assert f & ozk.OZK_FLAG_SCHEME2_CHOSEN
        assert bool(f & ozk.OZK_FLAG_S_UNPROVEN) == (int(info[6]) > 20)
    else:
        assert not f & ozk.OZK_FLAG_SCHEME2_CHOSEN


def test_flags_are_per_context(ctx):
    other = ozk.Context(0)
    A = synth.phi_matrix(20, 20, 1.0, 50)
    A[0, 0] = np.inf
    ozk.ozk_dgemm(other, ozk.OZK_SCHEME1, 3, dev(A), dev(A))
    assert ozk.ozk_get_flags(ctx) == 0
    assert ozk.ozk_get_flags(other) == ozk.OZK_FLAG_NONFINITE
    other.close()
