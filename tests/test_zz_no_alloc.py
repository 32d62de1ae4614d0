"""The allocation-free entry point ozk_dgemm_noalloc (the library's fixed
device buffer in place of a workspace) against ozk_dgemm, bit for bit, on
two calls in a row with the second smaller (the buffer keeps the first
call's contents), for both schemes, a long-K Scheme I call that folds K
runs, and the size limit."""
import numpy as np
import pytest

import oracle
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


def pair(M, N, K, seed):
    A = torch.from_numpy(synth.phi_matrix(M, K, 1.0, seed)).cuda()
    B = torch.from_numpy(synth.phi_matrix(K, N, 1.0, seed + 1)).cuda()
    return A, B


@pytest.mark.parametrize("scheme,count", [(ozk.OZK_SCHEME1, 7), (ozk.OZK_SCHEME1, 3), (ozk.OZK_SCHEME2, 12)])
def test_noalloc_matches_dgemm_on_two_calls(ctx, scheme, count):
    for (M, N, K), seed in (((700, 530, 1100), 11), ((300, 200, 260), 12)):
        print("case noalloc scheme %d count %d %dx%dx%d" % (scheme, count, M, N, K), flush=True)
        A, B = pair(M, N, K, seed)
        C0 = torch.from_numpy(synth.phi_matrix(M, N, 1.0, seed + 2)).cuda()
        want = ozk.ozk_dgemm(ctx, scheme, count, A, B, C=C0.clone(), alpha=0.75, beta=-1.5)
        got = ozk.ozk_dgemm_noalloc(ctx, scheme, count, A, B, C=C0.clone(), alpha=0.75, beta=-1.5)
        torch.cuda.synchronize()
        assert torch.equal(got, want)
        plain = ozk.ozk_dgemm_noalloc(ctx, scheme, count, A, B)
        torch.cuda.synchronize()
        An, Bn = A.cpu().numpy(), B.cpu().numpy()
        if scheme == ozk.OZK_SCHEME1:
            ref = oracle.s1_dgemm(An, Bn, count)
        else:
            from oracle import scheme2 as s2
            ref = s2.s2_dgemm(An, Bn, count)
        assert np.array_equal(plain.cpu().numpy(), ref)


def test_noalloc_long_k_fold(ctx):
    """K split into runs of 64 (the exact 128-bit fold of the partial sums
    lives in the fixed buffer too), then a call without the split."""
    ozk.ozk_set_k_split(ctx, 64)
    A, B = pair(130, 90, 300, 21)
    want = ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME1, 5, A, B)
    got = ozk.ozk_dgemm_noalloc(ctx, ozk.OZK_SCHEME1, 5, A, B)
    torch.cuda.synchronize()
    assert torch.equal(got, want)
    assert np.array_equal(got.cpu().numpy(), oracle.s1_dgemm(A.cpu().numpy(), B.cpu().numpy(), 5))
    ozk.ozk_set_k_split(ctx, 0)
    A, B = pair(64, 48, 100, 22)
    got = ozk.ozk_dgemm_noalloc(ctx, ozk.OZK_SCHEME1, 5, A, B)
    torch.cuda.synchronize()
    assert torch.equal(got, ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME1, 5, A, B))


def test_noalloc_rejects_problems_beyond_the_buffer(ctx):
    n = 4096  # Scheme I p = 7 needs 2 * 7 * 4096^2 bytes of packed slices, past 64 MiB
    assert ozk.ozk_workspace_size(ctx, ozk.OZK_OP_DGEMM, ozk.OZK_SCHEME1, n, n, n, 7) > ozk.OZK_NOALLOC_SCRATCH_BYTES
    A = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    C = torch.full((n, n), 3.0, dtype=torch.float64, device="cuda")
    with pytest.raises(ozk.OzkError) as ei:
        ozk.ozk_dgemm_noalloc(ctx, ozk.OZK_SCHEME1, 7, A, A, C=C)
    assert ei.value.status == ozk.OZK_ERR_WORKSPACE
    torch.cuda.synchronize()
    assert bool((C == 3.0).all())  # nothing was enqueued
    n = 2048  # the largest square Scheme I p = 7 problem that fits
    assert ozk.ozk_workspace_size(ctx, ozk.OZK_OP_DGEMM, ozk.OZK_SCHEME1, n, n, n, 7) <= ozk.OZK_NOALLOC_SCRATCH_BYTES
    A, B = pair(n, n, n, 31)
    got = ozk.ozk_dgemm_noalloc(ctx, ozk.OZK_SCHEME1, 7, A, B)
    torch.cuda.synchronize()
    assert torch.equal(got, ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME1, 7, A, B))
