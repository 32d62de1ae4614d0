"""Batched uneven problems in one launch per step (persistent GEMM), through
the C ABI: every problem of a batch equals its single-call result and the
CPU oracle bit for bit, and graph replays are bit-identical to the eager
run, also with eager work in between."""
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


def make_batch(count, lo, hi, seed, cplx):
    dims = synth.log_uniform_ints(3 * count, lo, hi, seed).reshape(count, 3)
    probs = []
    for i, (M, N, K) in enumerate(dims):
        M, N, K = int(M), int(N), int(K)
        if cplx:
            A = synth.complex_phi_matrix(M, K, 1.0, seed + 10 * i, seed + 10 * i + 1)
            B = synth.complex_phi_matrix(K, N, 1.0, seed + 10 * i + 2, seed + 10 * i + 3)
        else:
            A = synth.phi_matrix(M, K, 1.0, seed + 10 * i)
            B = synth.phi_matrix(K, N, 1.0, seed + 10 * i + 2)
        probs.append((A, B))
    return probs


@pytest.mark.parametrize("cplx,s", [(True, 16), (True, 7), (False, 14), (False, 1), (True, 20)])
def test_batch_matches_single_calls_and_oracle(ctx, cplx, s):
    probs = make_batch(12, 1, 300, 77 + s, cplx)
    probs.append((np.zeros((0, 5), probs[0][0].dtype), np.zeros((5, 3), probs[0][0].dtype)))  # empty M
    probs.append((np.zeros((70, 0), probs[0][0].dtype), np.zeros((0, 9), probs[0][0].dtype)))  # empty K
    dA = [dev(A) for A, _ in probs]
    dB = [dev(B) for _, B in probs]
    dtype = torch.complex128 if cplx else torch.float64
    dC = [torch.full((A.shape[0], B.shape[1]), float("nan"), dtype=dtype, device="cuda:0") for A, B in probs]
    op = ozk.OZK_OP_ZGEMM if cplx else ozk.OZK_OP_DGEMM
    plan = ozk.BatchPlan(ctx, op, ozk.OZK_SCHEME2, s, list(zip(dA, dB, dC)))
    plan.run()
    for i, (A, B) in enumerate(probs):
        got = host(dC[i])
        if cplx:
            single = host(ozk.ozk_zgemm_3m(ctx, s, dA[i], dB[i]))
        else:
            single = host(ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME2, s, dA[i], dB[i]))
        assert np.array_equal(got, single), i
        if i < 5 and A.size and B.size:
            ref = s2.z3m_gemm(A, B, s) if cplx else s2.s2_dgemm(A, B, s)
            assert np.array_equal(got, ref), i
    plan.close()


def test_batch_alpha_beta(ctx):
    s = 12
    probs = make_batch(5, 10, 90, 5, True)
    dA = [dev(A) for A, _ in probs]
    dB = [dev(B) for _, B in probs]
    C0 = [synth.complex_phi_matrix(A.shape[0], B.shape[1], 1.0, 300 + i, 400 + i) for i, (A, B) in enumerate(probs)]
    dC = [dev(c) for c in C0]
    al, be = 0.25 + 1j, -0.5 + 0.125j
    plan = ozk.BatchPlan(ctx, ozk.OZK_OP_ZGEMM, ozk.OZK_SCHEME2, s, list(zip(dA, dB, dC)), alpha=al, beta=be)
    plan.run()
    for i, (A, B) in enumerate(probs):
        assert np.array_equal(host(dC[i]), s2.z3m_gemm(A, B, s, alpha=al, beta=be, C=C0[i])), i
    plan.close()



@pytest.mark.parametrize("cplx", [False, True])
def test_batch_long_k_and_split_problems(ctx, cplx):
    """The two item schedules the plan can give a problem: K beyond one INT32
    run (more than 4095 chunks of 32 per modulus: the item walks each
    modulus as its own runs) next to a short-K problem, and a batch of one
    problem whose output tiles are cut into chunks for all eight XCD queues;
    both equal the single calls and the oracle on sampled rows and columns."""
    s = 3
    rng = np.random.default_rng(11)
    if cplx:
        A0 = synth.complex_phi_matrix(20, 131104, 1.0, 61, 62)
        B0 = synth.complex_phi_matrix(131104, 12, 1.0, 63, 64)
        A1 = synth.complex_phi_matrix(70, 96, 1.0, 65, 66)
        B1 = synth.complex_phi_matrix(96, 50, 1.0, 67, 68)
        A2 = synth.complex_phi_matrix(512, 64, 1.0, 69, 70)
        B2 = synth.complex_phi_matrix(64, 520, 1.0, 71, 72)
    else:
        A0 = synth.phi_matrix(20, 131104, 1.0, 61)
        B0 = synth.phi_matrix(131104, 12, 1.0, 63)
        A1 = synth.phi_matrix(70, 96, 1.0, 65)
        B1 = synth.phi_matrix(96, 50, 1.0, 67)
        A2 = synth.phi_matrix(512, 64, 1.0, 69)
        B2 = synth.phi_matrix(64, 520, 1.0, 71)
    op = ozk.OZK_OP_ZGEMM if cplx else ozk.OZK_OP_DGEMM
    for probs in ([(A0, B0), (A1, B1)], [(A2, B2)]):
        dA, dB, dC = _device_batch(probs)
        plan = ozk.BatchPlan(ctx, op, ozk.OZK_SCHEME2, s, list(zip(dA, dB, dC)))
        plan.run()
        for i, (A, B) in enumerate(probs):
            got = host(dC[i])
            single = host(ozk.ozk_zgemm_3m(ctx, s, dA[i], dB[i]) if cplx
                          else ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME2, s, dA[i], dB[i]))
            assert np.array_equal(got, single), i
            rows = np.sort(rng.choice(A.shape[0], size=min(6, A.shape[0]), replace=False))
            cols = np.sort(rng.choice(B.shape[1], size=min(5, B.shape[1]), replace=False))
            # the row and column scales depend only on their own row or column,
            # so the product of the sampled rows and columns is the full
            # product's values there
            ref = (s2.z3m_gemm(A[rows], B[:, cols], s) if cplx else s2.s2_dgemm(A[rows], B[:, cols], s))
            assert np.array_equal(got[np.ix_(rows, cols)], ref), i
        plan.close()

@pytest.mark.parametrize("cplx", [False, True])
def test_batch_exponent_cache_boundaries(ctx, cplx):
    """The batched row and column scale passes keep the entry exponents in
    LDS for short K (rows up to K = 1024; columns up to 512 real, 1024
    complex) and read the operand again beyond: problems on both sides of
    each boundary, with zero and tiny entries, equal the single calls and the
    oracle on sampled rows and columns."""
    s = 5
    rng = np.random.default_rng(23)
    probs = []
    for i, K in enumerate((511, 512, 513, 1023, 1024, 1025)):
        M, N = 33 + 7 * i, 41 + 5 * i
        if cplx:
            A = synth.complex_phi_matrix(M, K, 1.0, 300 + i, 310 + i)
            B = synth.complex_phi_matrix(K, N, 1.0, 320 + i, 330 + i)
        else:
            A = synth.phi_matrix(M, K, 1.0, 300 + i)
            B = synth.phi_matrix(K, N, 1.0, 320 + i)
        A[1, ::3] = 0
        A[2, 5] *= 1e-200
        B[::4, 3] = 0
        B[7, 4] *= 1e-200
        probs.append((A, B))
    dA, dB, dC = _device_batch(probs)
    op = ozk.OZK_OP_ZGEMM if cplx else ozk.OZK_OP_DGEMM
    plan = ozk.BatchPlan(ctx, op, ozk.OZK_SCHEME2, s, list(zip(dA, dB, dC)))
    plan.run()
    for i, (A, B) in enumerate(probs):
        got = host(dC[i])
        single = host(ozk.ozk_zgemm_3m(ctx, s, dA[i], dB[i]) if cplx
                      else ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME2, s, dA[i], dB[i]))
        assert np.array_equal(got, single), i
        rows = np.unique(np.concatenate([[1, 2], rng.choice(A.shape[0], size=4, replace=False)]))
        cols = np.unique(np.concatenate([[3, 4], rng.choice(B.shape[1], size=4, replace=False)]))
        ref = (s2.z3m_gemm(A[rows], B[:, cols], s) if cplx else s2.s2_dgemm(A[rows], B[:, cols], s))
        assert np.array_equal(got[np.ix_(rows, cols)], ref), i
    plan.close()


def test_batch_graph_replay_is_bit_identical(ctx):
    s = 16
    probs = make_batch(40, 16, 256, 123, True)
    dA = [dev(A) for A, _ in probs]
    dB = [dev(B) for _, B in probs]
    dC = [torch.zeros((A.shape[0], B.shape[1]), dtype=torch.complex128, device="cuda:0") for A, B in probs]
    plan = ozk.BatchPlan(ctx, ozk.OZK_OP_ZGEMM, ozk.OZK_SCHEME2, s, list(zip(dA, dB, dC)))
    plan.run()
    eager = [host(c).copy() for c in dC]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        plan.run(stream=side)  # warm up on the capture stream
        torch.cuda.synchronize()
        for c in dC:
            c.zero_()
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=side):
            plan.run(stream=side)
    torch.cuda.current_stream().wait_stream(side)
    for rep in range(3):
        for c in dC:
            c.fill_(complex(rep + 7.0, -1.0))  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i, c in enumerate(dC):
            assert np.array_equal(host(c), eager[i]), (rep, i)
    plan.close()


def test_batch_config_256_uneven_zgemm(ctx):
    """The batch workload: 256 ZGEMMs with M, N, K log-uniform in [64, 1024],
    one launch per step; sampled problems against single calls."""
    s = 16
    count = 256
    dims = synth.log_uniform_ints(3 * count, 64, 1024, synth.seed_for(4, 256, 1.0, 0)).reshape(count, 3)
    dA, dB, dC = [], [], []
    g = torch.Generator(device="cpu").manual_seed(9)
    for (M, N, K) in dims:
        M, N, K = int(M), int(N), int(K)
        a = (torch.rand((M, K), generator=g, dtype=torch.float64) - 0.5) + 1j * (
            torch.rand((M, K), generator=g, dtype=torch.float64) - 0.5)
        b = (torch.rand((K, N), generator=g, dtype=torch.float64) - 0.5) + 1j * (
            torch.rand((K, N), generator=g, dtype=torch.float64) - 0.5)
        dA.append(a.to("cuda:0"))
        dB.append(b.to("cuda:0"))
        dC.append(torch.empty((M, N), dtype=torch.complex128, device="cuda:0"))
    plan = ozk.BatchPlan(ctx, ozk.OZK_OP_ZGEMM, ozk.OZK_SCHEME2, s, list(zip(dA, dB, dC)))
    plan.run()
    torch.cuda.synchronize()
    tiles = plan.tiles()
    assert 0 < sum(tiles) < count  # both tiles in use
    for i in range(count):
        assert torch.equal(dC[i], ozk.ozk_zgemm_3m(ctx, s, dA[i], dB[i])), i
    plan.close()


def _device_batch(probs):
    dA = [dev(A) for A, _ in probs]
    dB = [dev(B) for _, B in probs]
    dtype = dA[0].dtype
    dC = [torch.full((A.shape[0], B.shape[1]), float("nan"), dtype=dtype, device="cuda:0") for A, B in probs]
    return dA, dB, dC


@pytest.mark.parametrize("cplx", [False, True])
def test_batch_tiles_from_the_table_are_bit_identical(cplx):
    """Every problem on the small tile, every problem on the large tile (the
    table entries of the batched op code decide), and the default choice:
    the same results as the single calls."""
    s = 10
    probs = make_batch(14, 30, 420, 900 + int(cplx), cplx)
    dA, dB, dC = _device_batch(probs)
    op = ozk.OZK_OP_ZGEMM if cplx else ozk.OZK_OP_DGEMM
    bop = ozk.OZK_OP_ZGEMM_BATCHED if cplx else ozk.OZK_OP_DGEMM_BATCHED
    singles = []
    ctx = ozk.Context(0)
    try:
        for i in range(len(probs)):
            singles.append(host(ozk.ozk_zgemm_3m(ctx, s, dA[i], dB[i]) if cplx else
                                ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME2, s, dA[i], dB[i])))
        default = ozk.BatchPlan(ctx, op, ozk.OZK_SCHEME2, s, list(zip(dA, dB, dC)))
        expect = [int(A.shape[0] >= 256 and B.shape[1] >= 256) for A, B in probs]
        assert default.tiles() == expect
        default.close()
        for kind in (0, 1):
            for A, B in probs:
                ozk.ozk_config_set(ctx, bop, ozk.OZK_SCHEME2, s, A.shape[0], B.shape[1], A.shape[1], (kind, 0, 4, 1))
            plan = ozk.BatchPlan(ctx, op, ozk.OZK_SCHEME2, s, list(zip(dA, dB, dC)))
            assert plan.tiles() == [kind] * len(probs)
            for c in dC:
                c.fill_(float("nan"))
            plan.run()
            for i in range(len(probs)):
                assert np.array_equal(host(dC[i]), singles[i]), (kind, i)
            plan.close()
        with pytest.raises(ozk.OzkError):  # batch tiles are 0 or 1
            ozk.ozk_config_set(ctx, bop, ozk.OZK_SCHEME2, s, 64, 64, 64, (2, 0, 4, 1))
    finally:
        ctx.close()


def test_tune_batch_picks_tiles_and_stores_them():
    s = 16
    probs = make_batch(24, 40, 700, 950, True)
    dA, dB, dC = _device_batch(probs)
    ctx = ozk.Context(0)
    try:
        plan = ozk.BatchPlan(ctx, ozk.OZK_OP_ZGEMM, ozk.OZK_SCHEME2, s, list(zip(dA, dB, dC)))
        plan.tune(reps=2)
        tiles = plan.tiles()
        for i, (A, B) in enumerate(probs):
            assert np.array_equal(host(dC[i]), host(ozk.ozk_zgemm_3m(ctx, s, dA[i], dB[i]))), i
            cfg, found, ms = ozk.ozk_config_get(ctx, ozk.OZK_OP_ZGEMM_BATCHED, ozk.OZK_SCHEME2, s, A.shape[0],
                                                B.shape[1], A.shape[1])
            assert found and cfg[0] == tiles[i] and ms > 0, (i, cfg, tiles[i])
        again = ozk.BatchPlan(ctx, ozk.OZK_OP_ZGEMM, ozk.OZK_SCHEME2, s, list(zip(dA, dB, dC)))
        assert again.tiles() == tiles  # a new plan of the context takes the tuned tiles
        for c in dC:
            c.fill_(float("nan"))
        again.run()
        for i in range(len(probs)):
            assert np.array_equal(host(dC[i]), host(ozk.ozk_zgemm_3m(ctx, s, dA[i], dB[i]))), i
        again.close()
        plan.close()
    finally:
        ctx.close()
