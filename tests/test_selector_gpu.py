"""The learned slice / modulus count selector through the C ABI: the device
exponent statistics and the a-priori bounds equal the oracle's exactly, the
network's decision follows the oracle's rule, the training kernels (MLP
forward, gradient, Adam) agree with the fp64 oracle to float32 accuracy,
ozk_dgemm_auto is bit-identical to ozk_dgemm at the scheme and count it
chose, and with the shipped parameters it never misses the tolerance on fresh
problems (judged by the CPU oracle's double-double product) while using
fewer slices and moduli than the bounds alone."""
import ctypes
import math
import os

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


def select(ctx, A, B, tol):
    M, K = A.shape
    N = B.shape[1]
    e = torch.empty(max(M, 1), dtype=torch.int32, device="cuda:0")
    f = torch.empty(max(N, 1), dtype=torch.int32, device="cuda:0")
    cnt = torch.empty(ozk.OZK_SELECTOR_COUNTERS, dtype=torch.int32, device="cuda:0")
    info = torch.empty(ozk.OZK_SELECTOR_INFO, dtype=torch.int32, device="cuda:0")
    feat = torch.empty(34, dtype=torch.float32, device="cuda:0")
    st = ozk.library().ozk_select(ctx.handle, tol, M, N, K, A.data_ptr(), ozk._ld(A), B.data_ptr(), ozk._ld(B),
                                  e.data_ptr(), f.data_ptr(), cnt.data_ptr(), info.data_ptr(), feat.data_ptr(),
                                  ozk._stream(None))
    ozk._check("ozk_select", st, ctx)
    return host(e)[:M], host(f)[:N], host(cnt), host(info), host(feat)


def check_decision(info, p_eff, s_eff=None):
    """Scheme I with p_eff slices when p_eff <= 8, else Scheme II with s_eff
    moduli (default: the bound's count; 20 when none is proven enough)."""
    if p_eff <= 8:
        assert info[4] == 1 and info[0] == max(p_eff, 1) and info[5] == 0, info.tolist()
    else:
        s_eff = info[6] if s_eff is None else s_eff
        assert info[4] == 2 and info[0] == 0 and info[5] == min(s_eff, 20), info.tolist()


def load_params(ctx, flat, threshold=0.5, margin=0):
    arr = (ctypes.c_float * len(flat))(*[float(x) for x in flat])
    thr = np.broadcast_to(np.asarray(threshold, np.float32), (ozk.OZK_SELECTOR_HEADS,))
    tarr = (ctypes.c_float * ozk.OZK_SELECTOR_HEADS)(*[float(x) for x in thr])
    st = ozk.library().ozk_selector_load(ctx.handle, ctypes.cast(arr, ctypes.c_void_p), len(flat),
                                         ctypes.cast(tarr, ctypes.c_void_p), margin)
    ozk._check("ozk_selector_load", st, ctx)


def oracle_params(flat):
    """Split the flat float32 parameter vector into the oracle's tuple."""
    flat = np.asarray(flat, np.float64)
    shapes = [(34, 64), (64,), (64, 64), (64,), (64, sel.N_OUT), (sel.N_OUT,)]
    out, o = [], 0
    for sh in shapes:
        n = int(np.prod(sh))
        out.append(flat[o:o + n].reshape(sh))
        o += n
    assert o == ozk.OZK_SELECTOR_PARAMS
    return tuple(out)


def random_flat(seed, scale=0.3):
    r = np.random.default_rng(seed)
    return (r.standard_normal(ozk.OZK_SELECTOR_PARAMS) * scale).astype(np.float32)


def dgemm_auto(ctx, tol, A, B, C=None, alpha=1.0, beta=0.0):
    M, K = A.shape
    N = B.shape[1]
    if C is None:
        C = torch.full((M, N), float("nan"), dtype=torch.float64, device="cuda:0")
    nb = ozk.ozk_workspace_size(ctx, ozk.OZK_OP_DGEMM, ozk.OZK_SCHEME1, M, N, K, 0)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda:0")
    info = torch.empty(ozk.OZK_SELECTOR_INFO, dtype=torch.int32, device="cuda:0")
    st = ozk.library().ozk_dgemm_auto(ctx.handle, tol, M, N, K, alpha, A.data_ptr(), ozk._ld(A), B.data_ptr(),
                                      ozk._ld(B), beta, C.data_ptr(), ozk._ld(C), ws.data_ptr(), nb,
                                      info.data_ptr(), ozk._stream(None))
    ozk._check("ozk_dgemm_auto", st, ctx)
    return C, host(info)


CASES = [(1, 1, 1, 0.5, 1), (37, 300, 45, 1.0, 2), (130, 77, 257, 3.0, 3), (64, 2048, 96, 0.0, 4),
         (5, 1000, 9, 6.0, 5)]


@pytest.mark.parametrize("M,K,N,phi,seed", CASES)
def test_statistics_and_bound_match_oracle(ctx, M, K, N, phi, seed):
    A = synth.phi_matrix(M, K, phi, seed)
    B = synth.phi_matrix(K, N, phi, seed + 100)
    if M > 2:
        A[1] = 0.0  # a zero row
        A[2, : K // 2] = 0.0
    for tol in (1e-5, 1e-9, 1e-13, 1e-16):
        e, f, cnt, info, feat = select(ctx, dev(A), dev(B), tol)
        assert np.array_equal(e, oracle.s1_row_exponents(A))
        assert np.array_equal(f, oracle.s1_col_exponents(B))
        ca, da = sel.deficit_counts(A, 1)
        cb, db = sel.deficit_counts(B, 0)
        assert cnt[:16].tolist() == ca.tolist() and cnt[16:32].tolist() == cb.tolist()
        assert cnt[32] == da and cnt[33] == db
        ref = sel.features(A, B, tol)
        assert np.allclose(feat, ref, rtol=1e-6, atol=1e-7), (feat, ref)
        assert info[2] == sel.p_bound(A, B, tol)
        assert info[6] == sel.s_bound(A, B, tol)
        assert info[1] == 0  # no network loaded in this context
        check_decision(info, info[2])


def test_nonfinite_lines_are_skipped(ctx):
    A = synth.phi_matrix(40, 70, 2.0, 9)
    B = synth.phi_matrix(70, 33, 2.0, 10)
    A[3, 5] = np.inf
    B[7, 2] = np.nan
    _, _, cnt, _, _ = select(ctx, dev(A), dev(B), 1e-10)
    assert cnt[:16].tolist() == sel.deficit_counts(A, 1)[0].tolist()
    assert cnt[16:32].tolist() == sel.deficit_counts(B, 0)[0].tolist()


def test_out_of_range_uses_the_bound(ctx):
    A = synth.phi_matrix(2, 16400, 0.5, 11)
    B = synth.phi_matrix(16400, 3, 0.5, 12)
    ctx2 = ozk.Context(0)
    try:
        load_params(ctx2, np.full(ozk.OZK_SELECTOR_PARAMS, 0.0, np.float32), 0.5, 0)  # p_net = s_net = 1
        _, _, _, info, _ = select(ctx2, dev(A), dev(B), 1e-10)
        assert info[3] == 1 and info[1] == 1 and info[7] == 1 and info[2] == sel.p_bound(A, B, 1e-10)
        check_decision(info, info[2])
        A2, B2 = A[:, :1000].copy(), B[:1000].copy()
        _, _, _, info, _ = select(ctx2, dev(A2), dev(B2), 1e-10)
        assert info[3] == 0 and info[4] == 1 and info[0] == 1  # in range: the network's choice
        _, _, _, info, _ = select(ctx2, dev(A2), dev(B2), 1e-17)  # tolerance outside the range
        assert info[3] == 1
        check_decision(info, info[2])
    finally:
        ctx2.close()


def test_network_decision_matches_oracle(ctx):
    """p_net, s_net and the (scheme, count) decision equal the oracle's rule
    for a random network, scalar and per-head thresholds and a margin."""
    flat = random_flat(5, 0.4)
    ctx2 = ozk.Context(0)
    per_head = np.linspace(0.2, 0.8, ozk.OZK_SELECTOR_HEADS).astype(np.float32)
    try:
        for thr, margin in ((0.5, 0), (0.3, 1), (per_head, 0)):
            load_params(ctx2, flat, thr, margin)
            for seed in range(8):
                A = synth.phi_matrix(50, 120, 0.5 * seed, 30 + seed)
                B = synth.phi_matrix(120, 40, 0.5 * seed, 40 + seed)
                tol = 10.0 ** -(6 + seed)
                _, _, _, info, feat = select(ctx2, dev(A), dev(B), tol)
                logits, _ = sel.mlp_forward(oracle_params(flat), feat.astype(np.float64).reshape(1, -1))
                z = logits[0]
                if np.min(np.abs(1.0 / (1.0 + np.exp(-z)) - thr)) < 1e-4:
                    continue  # too close to a threshold to decide in float32
                p_net, s_net = (int(v[0]) for v in sel.predict(logits, thr, margin))
                assert info[1] == p_net and info[7] == s_net, (info.tolist(), p_net, s_net)
                assert info[6] == sel.s_bound(A, B, tol)
                scheme, count = sel.decide(p_net, s_net, int(info[2]), int(info[6]), not info[3])
                assert info[4] == scheme and (info[0] if scheme == 1 else info[5]) == count, info.tolist()
    finally:
        ctx2.close()


def test_mlp_forward_matches_oracle(ctx):
    flat = random_flat(1)
    r = np.random.default_rng(2)
    X = r.random((300, 34)).astype(np.float32)
    out = torch.empty((300, sel.N_OUT), dtype=torch.float32, device="cuda:0")
    w, x = dev(flat), dev(X)
    st = ozk.library().ozk_mlp_forward(ctx.handle, w.data_ptr(), x.data_ptr(), 300, out.data_ptr(),
                                       ozk._stream(None))
    ozk._check("ozk_mlp_forward", st, ctx)
    ref, _ = sel.mlp_forward(oracle_params(flat), X.astype(np.float64))
    assert np.allclose(host(out), ref, rtol=1e-4, atol=1e-4 * np.abs(ref).max())


def test_mlp_grad_and_adam_match_oracle(ctx):
    flat = random_flat(3)
    r = np.random.default_rng(4)
    n = 257
    X = r.random((n, 34)).astype(np.float32)
    Y = sel.ordinal_targets(r.integers(1, 10, n), r.integers(1, 22, n)).astype(np.float32)
    w, x, y = dev(flat), dev(X), dev(Y)
    g = torch.empty(ozk.OZK_SELECTOR_PARAMS, dtype=torch.float32, device="cuda:0")
    loss = torch.empty(1, dtype=torch.float32, device="cuda:0")
    lib = ozk.library()
    st = lib.ozk_mlp_grad(ctx.handle, w.data_ptr(), x.data_ptr(), y.data_ptr(), n, g.data_ptr(), loss.data_ptr(),
                          ozk._stream(None))
    ozk._check("ozk_mlp_grad", st, ctx)
    P = oracle_params(flat)
    logits, cache = sel.mlp_forward(P, X.astype(np.float64))
    ref_loss = sel.bce_loss(logits, Y.astype(np.float64))
    grads = np.concatenate([q.reshape(-1) for q in sel.mlp_backward(P, cache, logits, Y.astype(np.float64))])
    assert abs(float(host(loss)[0]) - ref_loss) <= 1e-5 * abs(ref_loss)
    gg = host(g)
    assert np.allclose(gg, grads, rtol=1e-3, atol=1e-4 * np.abs(grads).max())
    # two Adam steps from zero moments
    m = torch.zeros_like(g)
    v = torch.zeros_like(g)
    pm = tuple(np.zeros_like(q) for q in P)
    pv = tuple(np.zeros_like(q) for q in P)
    gt = tuple(np.asarray(q, np.float64) for q in oracle_params(gg))
    cur = P
    for step in (1, 2):
        st = lib.ozk_mlp_adam(ctx.handle, w.data_ptr(), g.data_ptr(), m.data_ptr(), v.data_ptr(), step, 1e-2,
                              ozk._stream(None))
        ozk._check("ozk_mlp_adam", st, ctx)
        cur, pm, pv = sel.adam_step(cur, gt, pm, pv, step, lr=1e-2)
    ref = np.concatenate([q.reshape(-1) for q in cur])
    assert np.allclose(host(w), ref, rtol=1e-5, atol=1e-5)


def test_ref_dd_against_exact_sums(ctx):
    from fractions import Fraction
    A = synth.phi_matrix(6, 200, 3.0, 50)
    B = synth.phi_matrix(200, 5, 3.0, 51)
    rows = torch.tensor([0, 5, 3, 2, 7, -1], dtype=torch.int64, device="cuda:0")
    cols = torch.tensor([0, 4, 1, 2, 0, 0], dtype=torch.int64, device="cuda:0")
    n = rows.numel()
    hi = torch.empty(n, dtype=torch.float64, device="cuda:0")
    lo = torch.empty_like(hi)
    ab = torch.empty_like(hi)
    dA, dB = dev(A), dev(B)
    st = ozk.library().ozk_ref_dd(ctx.handle, 6, 5, 200, dA.data_ptr(), 200, dB.data_ptr(), 5, n, rows.data_ptr(),
                                  cols.data_ptr(), hi.data_ptr(), lo.data_ptr(), ab.data_ptr(), ozk._stream(None))
    ozk._check("ozk_ref_dd", st, ctx)
    h, l, a = host(hi), host(lo), host(ab)
    for idx, (i, j) in enumerate(zip(host(rows), host(cols))):
        if not (0 <= i < 6 and 0 <= j < 5):
            assert math.isnan(h[idx]) and math.isnan(l[idx]) and math.isnan(a[idx])
            continue
        exact = sum(Fraction(float(A[i, k])) * Fraction(float(B[k, j])) for k in range(200))
        absab = sum(abs(float(A[i, k]) * float(B[k, j])) for k in range(200))
        err = abs(Fraction(float(h[idx])) + Fraction(float(l[idx])) - exact)
        assert float(err) <= 200 * 2.0 ** -100 * absab
        assert abs(a[idx] - absab) <= 1e-13 * absab


@pytest.mark.parametrize("M,K,N,phi", [(33, 130, 71, 1.0), (256, 512, 300, 2.5), (1, 7, 1, 0.0)])
def test_dgemm_auto_equals_dgemm_at_chosen_p(ctx, M, K, N, phi):
    A = synth.phi_matrix(M, K, phi, 60)
    B = synth.phi_matrix(K, N, phi, 61)
    C0 = synth.phi_matrix(M, N, 1.0, 62)
    dA, dB = dev(A), dev(B)
    ctx2 = ozk.Context(0)
    try:
        load_params(ctx2, random_flat(7, 0.5), 0.5, 0)
        for tol in (1e-6, 1e-10, 1e-14):
            for c in (ctx, ctx2):
                C, info = dgemm_auto(c, tol, dA, dB, dev(C0), alpha=0.75, beta=-0.5)
                scheme, p, s = int(info[4]), int(info[0]), int(info[5])
                if scheme == 1:
                    assert 1 <= p <= 8
                    ref = ozk.ozk_dgemm(c, ozk.OZK_SCHEME1, p, dA, dB, dev(C0), alpha=0.75, beta=-0.5)
                    expect = oracle.s1_dgemm(A, B, p, alpha=0.75, beta=-0.5, C=C0)
                else:
                    assert scheme == 2 and 1 <= s <= 20
                    ref = ozk.ozk_dgemm(c, ozk.OZK_SCHEME2, s, dA, dB, dev(C0), alpha=0.75, beta=-0.5)
                    expect = s2.s2_dgemm(A, B, s, alpha=0.75, beta=-0.5, C=C0)
                assert torch.equal(C, ref), (tol, info.tolist())
                if M * N * K <= 40000:
                    assert np.array_equal(host(C), expect)
    finally:
        ctx2.close()


def test_dgemm_auto_takes_scheme2_when_scheme1_cannot(ctx):
    """A wide exponent range and a tight tolerance: no slice count up to 8 is
    proven enough, so the modulus count of the Scheme II bound is used; the
    result is bit-identical to Scheme II at that s and to the oracle, and it
    meets the tolerance whenever the bound proved that s enough."""
    A = synth.phi_matrix(45, 90, 3.0, 91)
    B = synth.phi_matrix(90, 30, 3.0, 92)
    dA, dB = dev(A), dev(B)
    hi, lo = oracle.gemm_dd(A, B)
    seen = False
    for tol in (1e-8, 1e-11, 1e-14):
        if sel.p_bound(A, B, tol) <= 8:
            continue
        seen = True
        C, info = dgemm_auto(ctx, tol, dA, dB)
        sb = sel.s_bound(A, B, tol)
        assert info[4] == 2 and info[0] == 0 and info[6] == sb and info[5] == min(sb, 20), info.tolist()
        s = int(info[5])
        got = host(C)
        assert np.array_equal(got, host(ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME2, s, dA, dB)))
        assert np.array_equal(got, s2.s2_dgemm(A, B, s))
        if sb <= 20:
            assert oracle.metrics.e_cw(got, hi, lo, A, B) <= tol
    assert seen  # the inputs do leave Scheme I unproven at some tolerance


def test_dgemm_auto_long_k_folds(ctx):
    """K beyond the p = 8 run length: the K runs fold exactly at any chosen p."""
    K = ozk.ozk_s1_k_split(8) + 100
    A = synth.phi_matrix(3, K, 0.5, 70)
    B = synth.phi_matrix(K, 2, 0.5, 71)
    dA, dB = dev(A), dev(B)
    C, info = dgemm_auto(ctx, 1e-12, dA, dB)
    if info[4] == 1:
        assert torch.equal(C, ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME1, int(info[0]), dA, dB))
    else:
        assert torch.equal(C, ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME2, int(info[5]), dA, dB))


def test_dgemm_auto_graph_replay(ctx):
    A = synth.phi_matrix(200, 300, 1.5, 80)
    B = synth.phi_matrix(300, 150, 1.5, 81)
    dA, dB = dev(A), dev(B)
    C = torch.zeros((200, 150), dtype=torch.float64, device="cuda:0")
    nb = ozk.ozk_workspace_size(ctx, ozk.OZK_OP_DGEMM, ozk.OZK_SCHEME1, 200, 150, 300, 0)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda:0")
    info = torch.zeros(ozk.OZK_SELECTOR_INFO, dtype=torch.int32, device="cuda:0")
    lib = ozk.library()

    def run(stream):
        st = lib.ozk_dgemm_auto(ctx.handle, 1e-11, 200, 150, 300, 1.0, dA.data_ptr(), 300, dB.data_ptr(), 150, 0.0,
                                C.data_ptr(), 150, ws.data_ptr(), nb, info.data_ptr(), stream.cuda_stream)
        ozk._check("ozk_dgemm_auto", st, ctx)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        run(side)
        torch.cuda.synchronize()
        eager = host(C).copy()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            run(side)
    torch.cuda.current_stream().wait_stream(side)
    for rep in range(3):
        C.fill_(float(rep) + 3.0)
        info.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(C), eager), rep
        i = host(info)
        assert (i[4] == 1 and 1 <= i[0] <= 8) or (i[4] == 2 and 1 <= i[5] <= 20)


def test_invalid_arguments(ctx):
    lib = ozk.library()
    bad = (ctypes.c_float * 3)(1.0, 2.0, 3.0)
    thr = (ctypes.c_float * ozk.OZK_SELECTOR_HEADS)(*([0.5] * ozk.OZK_SELECTOR_HEADS))
    assert lib.ozk_selector_load(ctx.handle, ctypes.cast(bad, ctypes.c_void_p), 3, ctypes.cast(thr, ctypes.c_void_p),
                                 0) == ozk.OZK_ERR_INVALID_ARG
    good = (ctypes.c_float * ozk.OZK_SELECTOR_PARAMS)()
    thr[5] = 1.0  # thresholds must lie in (0, 1)
    assert lib.ozk_selector_load(ctx.handle, ctypes.cast(good, ctypes.c_void_p), ozk.OZK_SELECTOR_PARAMS,
                                 ctypes.cast(thr, ctypes.c_void_p), 0) == ozk.OZK_ERR_INVALID_ARG
    assert lib.ozk_last_arg(ctx.handle) == 4
    A = dev(synth.phi_matrix(4, 4, 1.0, 1))
    i32 = torch.empty(64, dtype=torch.int32, device="cuda:0")
    for tol in (0.0, -1.0, 1.0, float("nan")):
        st = lib.ozk_select(ctx.handle, tol, 4, 4, 4, A.data_ptr(), 4, A.data_ptr(), 4, i32.data_ptr(),
                            i32.data_ptr(), i32.data_ptr(), i32.data_ptr(), None, ozk._stream(None))
        assert st == ozk.OZK_ERR_INVALID_ARG and lib.ozk_last_arg(ctx.handle) == 2
    st = lib.ozk_dgemm_auto(ctx.handle, 1e-10, 4, 4, 4, 1.0, A.data_ptr(), 4, A.data_ptr(), 4, 0.0, A.data_ptr(), 4,
                            i32.data_ptr(), 16, None, ozk._stream(None))
    assert st == ozk.OZK_ERR_WORKSPACE


WEIGHTS = os.path.join(os.path.dirname(ozk.__file__), "selector_weights.json")


def trained_meta():
    from paper_2606_25453_amd import selector as train
    if not os.path.exists(WEIGHTS):
        return None
    d = train.load()
    return d if len(d.get("thresholds", ())) == ozk.OZK_SELECTOR_HEADS else None


@pytest.mark.skipif(trained_meta() is None, reason="no trained parameters of this network shape")
def test_trained_selector_never_misses_the_tolerance(ctx):
    """Fresh problems from the training distribution (M, N in [256, 4096], K
    in [256, 16384] log-uniform, phi_A, phi_B in [0, 4]; seeds outside the
    training and calibration sets) at four tolerances: whenever the decision
    is Scheme I, or Scheme II at a count the network or the bound chose below
    the proven maximum, the result meets the tolerance -- judged by the CPU
    oracle's double-double product on sampled outputs (an 24 x 24 block of
    rows and columns, the per-row and per-column scales make them exactly the
    full product's), and by the library's double-double kernel on every
    output of the smaller problems.  On average fewer slices and moduli are
    used than with the bounds alone."""
    from oracle import metrics
    from paper_2606_25453_amd import selector as train
    ctx2 = ozk.Context(0)
    try:
        train.install(ctx2)
        gen = torch.Generator(device="cuda:0").manual_seed(987654)
        used_p, bound_p, used_s, bound_s = [], [], [], []
        rng = np.random.default_rng(123457)
        for i in range(40):
            M, N = (int(v) for v in synth.log_uniform_ints(2, 256, 4096, 7000 + i))
            K = int(synth.log_uniform_ints(1, 256, 16384, 8000 + i)[0])
            phi_a, phi_b = (float(v) for v in rng.uniform(0.0, 4.0, 2))
            A, B = train.random_problem(gen, M, N, K, phi_a, phi_b, "cuda:0")
            rows = np.unique(np.concatenate([rng.integers(0, M, 22), [0, M - 1]]))
            cols = np.unique(np.concatenate([rng.integers(0, N, 22), [0, N - 1]]))
            r, c = torch.from_numpy(rows).cuda(), torch.from_numpy(cols).cuda()
            As, Bs = A.index_select(0, r).cpu().numpy(), B.index_select(1, c).cpu().numpy()
            hi, lo = oracle.gemm_dd(As, Bs)
            full = train.dd_reference(ctx2, A, B) if M * N <= (1 << 21) else None
            for tol in (1e-6, 1e-9, 1e-12, 1e-14):
                C, info = dgemm_auto(ctx2, tol, A, B)
                got = C.index_select(0, r).index_select(1, c).cpu().numpy()
                err = metrics.e_cw(got, hi, lo, As, Bs)
                err_full = train.e_cw(C, *full) if full is not None else 0.0
                proven = info[4] == 1 or info[6] <= 20
                case = (i, M, N, K, round(phi_a, 3), round(phi_b, 3), tol, info.tolist(), err, err_full)
                if proven:
                    assert err <= tol and err_full <= tol, case
                if info[3] == 0:  # in range: the network took part
                    used_p.append(int(info[0]) if info[4] == 1 else 9)
                    bound_p.append(min(int(info[2]), 9))
                    if info[4] == 2:
                        used_s.append(int(info[5]))
                        bound_s.append(min(int(info[6]), 20))
            del A, B, C
        assert np.mean(used_p) < np.mean(bound_p)
        if used_s:
            assert np.mean(used_s) <= np.mean(bound_s)
        print("mean p (9 = Scheme II) %.2f against %.2f for the bound; mean s %.2f against %.2f (%d in Scheme II)"
              % (np.mean(used_p), np.mean(bound_p), np.mean(used_s) if used_s else 0,
                 np.mean(bound_s) if bound_s else 0, len(used_s)), flush=True)
    finally:
        ctx2.close()


def test_trained_selector_at_the_headline_size(ctx):
    """8192^3, phi = 1 for both operands, at 1e-13 and 1e-10: the automatic
    call meets the tolerance on sampled outputs judged by the CPU oracle's
    double-double product, and picks a Scheme I slice count (the fixed-p
    calls show p = 7 meets 1e-13 there with room to spare)."""
    from oracle import metrics
    from paper_2606_25453_amd import selector as train
    n = 8192
    ctx2 = ozk.Context(0)
    try:
        train.install(ctx2)
        A = synth.phi_matrix_device(n, n, 1.0, 424242)
        B = synth.phi_matrix_device(n, n, 1.0, 434343)
        rng = np.random.default_rng(99)
        rows = np.unique(np.concatenate([rng.integers(0, n, 14), [0, n - 1]]))
        cols = np.unique(np.concatenate([rng.integers(0, n, 14), [0, n - 1]]))
        r, c = torch.from_numpy(rows).cuda(), torch.from_numpy(cols).cuda()
        As, Bs = A.index_select(0, r).cpu().numpy(), B.index_select(1, c).cpu().numpy()
        hi, lo = oracle.gemm_dd(As, Bs)
        for tol in (1e-13, 1e-10):
            C, info = dgemm_auto(ctx2, tol, A, B)
            got = C.index_select(0, r).index_select(1, c).cpu().numpy()
            err = metrics.e_cw(got, hi, lo, As, Bs)
            print("tol %g: scheme %d p %d (bound %d), E_cw %.3g" % (tol, info[4], info[0], info[2], err), flush=True)
            assert info[3] == 0 and info[4] == 1 and info[0] <= 8, info.tolist()
            assert err <= tol, (tol, info.tolist(), err)
            del C
    finally:
        ctx2.close()
