"""Argument checks of the binding and of the C ABI on the GPU: tensors of
the wrong dtype, shape or size are refused before anything is enqueued, the
Scheme II K limit is enforced, and the scales at that limit still match the
oracle."""
import numpy as np
import pytest

import oracle
import paper_2606_25453_amd as ozk
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


def test_bad_tensors_raise_before_launch(ctx):
    d = torch.device("cuda:0")
    A = torch.ones((8, 5), dtype=torch.float64, device=d)
    B = torch.ones((5, 6), dtype=torch.float64, device=d)
    C = torch.full((8, 6), 3.0, dtype=torch.float64, device=d)
    cases = [
        (lambda: ozk.ozk_dgemm(ctx, 1, 4, A, B, ws=torch.zeros(1 << 20, dtype=torch.float32, device=d)), "dtype"),
        (lambda: ozk.ozk_dgemm_auto(ctx, 1e-13, A, B, info=torch.zeros(8, dtype=torch.int64, device=d)), "dtype"),
        (lambda: ozk.ozk_dgemm_auto(ctx, 1e-13, A, B, info=torch.zeros(4, dtype=torch.int32, device=d)),
         "elements"),
        (lambda: ozk.ozk_dgemm(ctx, 1, 4, A, B.T.contiguous()), "inner dimensions"),
        (lambda: ozk.ozk_dgemm(ctx, 1, 4, A, B, C=C[:, :5]), "shape"),
        (lambda: ozk.ozk_dgemm(ctx, 1, 4, A.float(), B.float()), "dtype"),
        (lambda: ozk.ozk_zgemm_3m(ctx, 8, A, B), "dtype"),
        (lambda: ozk.ozk_s1_gemm(ctx, 3, 8, 6, 5, torch.zeros(10, dtype=torch.int8, device=d),
                                 torch.zeros(8, dtype=torch.int32, device=d),
                                 torch.zeros(1 << 20, dtype=torch.int8, device=d),
                                 torch.zeros(6, dtype=torch.int32, device=d), C), "elements"),
        (lambda: ozk.ozk_s1_split_rows(ctx, 3, A, e=torch.zeros(3, dtype=torch.int32, device=d)), "elements"),
        (lambda: ozk.ozk_s2_crt(ctx, 4, 8, 6, torch.zeros((4, 8, 6), dtype=torch.int8, device=d),
                                torch.zeros(8, dtype=torch.int32, device=d), torch.zeros(6, dtype=torch.int32, device=d),
                                C.to(torch.complex128)), "dtype"),
    ]
    for fn, what in cases:
        with pytest.raises(ValueError) as ei:
            fn()
        assert what in str(ei.value), (what, str(ei.value))
    torch.cuda.synchronize()
    assert bool((C == 3.0).all())  # nothing ran
    out = ozk.ozk_dgemm(ctx, 1, 4, A, B)
    torch.cuda.synchronize()
    assert bool((out == 5.0).all())


def test_scheme2_k_limit(ctx):
    """K above 2^22 is refused by every Scheme II entry point (the norm-bound
    sums would leave 64 bits); Scheme I takes it."""
    K = ozk.OZK_S2_MAX_K + 32
    d = torch.device("cuda:0")
    A = torch.zeros((1, K), dtype=torch.float64, device=d)
    B = torch.zeros((K, 1), dtype=torch.float64, device=d)
    ws = torch.empty(1 << 20, dtype=torch.uint8, device=d)
    for fn in (lambda: ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME2, 8, A, B, ws=ws),
               lambda: ozk.ozk_dgemm_t(ctx, ozk.OZK_SCHEME2, 8, A, B, ws=ws),
               lambda: ozk.ozk_s2_split_rows(ctx, 1, A),
               lambda: ozk.ozk_dgemm_auto(ctx, 1e-13, A, B, ws=ws)):
        with pytest.raises(ozk.OzkError) as ei:
            fn()
        assert ei.value.status == ozk.OZK_ERR_UNSUPPORTED
    out = ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME1, 2, A + 1.0, B + 0.5)
    torch.cuda.synchronize()
    assert float(out[0, 0]) == 0.5 * K


def test_scheme2_scales_at_the_k_limit(ctx):
    """At K = 2^22 every norm-bound sum reaches 2^62 and stays exact: row and
    column scales match the oracle, including a line of equal maximal
    entries (the closed form sigma = T - (e + 11))."""
    K = ozk.OZK_S2_MAX_K
    rng = np.random.default_rng(3)
    X = np.full((2, K), 0.75)
    X[1] = rng.uniform(-1, 1, K)
    ta, tb = s2.targets(1)
    sig_ref, _ = s2.row_scales(X, ta)
    assert int(sig_ref[0]) == ta - 11
    Xd = torch.from_numpy(X).to("cuda:0")
    sig, _ = ozk.ozk_s2_split_rows(ctx, 1, Xd)
    assert np.array_equal(sig.cpu().numpy()[:2], sig_ref)
    Y = np.ascontiguousarray(X.T)
    tau_ref, _ = s2.col_scales(Y, tb)
    tau, _ = ozk.ozk_s2_split_cols(ctx, 1, torch.from_numpy(Y).to("cuda:0"))
    assert np.array_equal(tau.cpu().numpy()[:2], tau_ref)
