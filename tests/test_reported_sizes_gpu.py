"""Oracle parity at every size and configuration whose throughput is
reported: the headline Scheme I DGEMM 8192^3 in the shipped tuned
configurations, Scheme I at 16384^3, Scheme II and 3M ZGEMM at 8192^3 and
16384^3, SGEMM at 16384^3, CGEMM at 4096^3, the unfused ablation at 8192^3,
and every raster configuration on a grid whose tile count is a multiple of 8
(the XCD-aware order).

Full-size inputs are drawn on the GPU with a seeded generator; the row
scales depend only on a row of A and the column scales only on a column of
B, so the oracle run on the sampled rows and columns computes exactly the
sampled outputs, which must match bit for bit.  Accuracy is measured on the
same samples against the oracle's double-double product."""
import itertools
import os

import numpy as np
import pytest

import oracle
import paper_2606_25453_amd as ozk
import synth
from oracle import metrics
from oracle import scheme2 as s2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SHIPPED = os.path.join(os.path.dirname(os.path.abspath(ozk.__file__)), "gemm_configs.json")


@pytest.fixture()
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = ozk.Context(0)
    yield c
    c.close()
    torch.cuda.empty_cache()


def real_pair(M, N, K, seed, dtype=torch.float64):
    A = synth.phi_matrix_device(M, K, 1.0, seed).to(dtype)
    B = synth.phi_matrix_device(K, N, 1.0, seed + 1).to(dtype)
    return A, B


def complex_pair(M, N, K, seed, dtype=torch.complex128):
    A = torch.complex(synth.phi_matrix_device(M, K, 1.0, seed), synth.phi_matrix_device(M, K, 1.0, seed + 2))
    B = torch.complex(synth.phi_matrix_device(K, N, 1.0, seed + 1), synth.phi_matrix_device(K, N, 1.0, seed + 3))
    return A.to(dtype), B.to(dtype)


def sample(n, k, seed):
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([rng.integers(0, n, k), [0, n - 1]]))


def sub(A, B, rows, cols):
    """Host copies of the sampled rows of A and columns of B."""
    r = torch.from_numpy(rows).to(A.device)
    c = torch.from_numpy(cols).to(B.device)
    return A.index_select(0, r).cpu().numpy(), B.index_select(1, c).cpu().numpy()


def block(C, rows, cols):
    r = torch.from_numpy(rows).to(C.device)
    c = torch.from_numpy(cols).to(C.device)
    torch.cuda.synchronize()
    return C.index_select(0, r).index_select(1, c).cpu().numpy()


def report(tag, got, native, As, Bs):
    """E_cw (the gate), E_nw, bits and the median relative error of the
    sampled block against the oracle's double-double product."""
    hi, lo = oracle.zgemm_dd(As, Bs) if np.iscomplexobj(As) else oracle.gemm_dd(As, Bs)
    out = {}
    for name, C in (("emulated", got), ("native", native)):
        cw = metrics.e_cw(C, hi, lo, As, Bs)
        out[name] = (cw, metrics.e_nw(C, hi, lo), metrics.bits(cw), metrics.median_rel(C, hi, lo))
    print("%s: E_cw %.3g (native %.3g), E_nw %.3g (native %.3g), bits %.1f, median rel %.3g" % (
        tag, out["emulated"][0], out["native"][0], out["emulated"][1], out["native"][1], out["emulated"][2],
        out["emulated"][3]), flush=True)
    return out["emulated"][0], out["native"][0]


@pytest.mark.parametrize("p,cfg", [(7, (1, 0, 2, 1)), (8, (0, 0, 2, 1)), (6, None)])
def test_headline_8192_in_shipped_configuration(ctx, p, cfg):
    n = 8192
    ozk.ozk_config_load(ctx, SHIPPED)
    got_cfg, found, _ = ozk.ozk_config_get(ctx, ozk.OZK_OP_DGEMM, ozk.OZK_SCHEME1, p, n, n, n)
    if cfg is not None:
        assert found and got_cfg == cfg  # the configuration the benchmark times
    print("case Scheme I %d^3 p=%d config %s" % (n, p, got_cfg), flush=True)
    A, B = real_pair(n, n, n, 8100 + p)
    C = ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME1, p, A, B)
    rows, cols = sample(n, 30, p), sample(n, 30, p + 100)
    As, Bs = sub(A, B, rows, cols)
    got = block(C, rows, cols)
    assert np.array_equal(got, oracle.s1_dgemm(As, Bs, p))
    nat = block(torch.matmul(A, B), rows, cols)
    err, err_nat = report("Scheme I 8192^3 p=%d" % p, got, nat, As, Bs)
    if p >= 7:
        assert err <= 1e-13
    if p == 8:
        assert err <= 2 * err_nat, (err, err_nat)


@pytest.mark.parametrize("p", [7, 8])
def test_scheme1_16384(ctx, p):
    n = 16384
    print("case Scheme I %d^3 p=%d" % (n, p), flush=True)
    A, B = real_pair(n, n, n, 16300 + p)
    C = ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME1, p, A, B)
    rows, cols = sample(n, 20, p), sample(n, 20, p + 1)
    As, Bs = sub(A, B, rows, cols)
    got = block(C, rows, cols)
    assert np.array_equal(got, oracle.s1_dgemm(As, Bs, p))
    nat = block(torch.matmul(A, B), rows, cols)
    err, _ = report("Scheme I 16384^3 p=%d" % p, got, nat, As, Bs)
    assert err <= 1e-13


def test_unfused_ablation_8192(ctx):
    n, p = 8192, 7
    print("case unfused Scheme I %d^3 p=%d" % (n, p), flush=True)
    A, B = real_pair(n, n, n, 8400)
    C = ozk.ozk_s1_dgemm_unfused(ctx, p, A, B)
    rows, cols = sample(n, 16, 1), sample(n, 16, 2)
    As, Bs = sub(A, B, rows, cols)
    assert np.array_equal(block(C, rows, cols), oracle.s1_dgemm(As, Bs, p))
    assert torch.equal(C, ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME1, p, A, B))


@pytest.mark.parametrize("M,N,K,s", [(16384, 16384, 16384, 15), (8192, 8192, 2048, 14), (8192, 8192, 2048, 16),
                                     (4096, 4096, 4096, 14), (4096, 4096, 4096, 16)])
def test_scheme2_reported(ctx, M, N, K, s):
    print("case Scheme II %dx%dx%d s=%d" % (M, N, K, s), flush=True)
    A, B = real_pair(M, N, K, 9000 + s)
    C = ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME2, s, A, B)
    rows, cols = sample(M, 16, s), sample(N, 16, s + 1)
    As, Bs = sub(A, B, rows, cols)
    got = block(C, rows, cols)
    assert np.array_equal(got, s2.s2_dgemm(As, Bs, s))
    nat = block(torch.matmul(A, B), rows, cols)
    report("Scheme II %dx%dx%d s=%d" % (M, N, K, s), got, nat, As, Bs)


@pytest.mark.parametrize("n,s", [(4096, 16), (8192, 16), (16384, 15)])
def test_zgemm_3m_reported(ctx, n, s):
    print("case 3M ZGEMM %d^3 s=%d" % (n, s), flush=True)
    A, B = complex_pair(n, n, n, 9500 + n // 1024 + s)
    C = ozk.ozk_zgemm_3m(ctx, s, A, B)
    rows, cols = sample(n, 12, s), sample(n, 12, s + 1)
    As, Bs = sub(A, B, rows, cols)
    got = block(C, rows, cols)
    assert np.array_equal(got, s2.z3m_gemm(As, Bs, s))
    nat = block(torch.matmul(A, B), rows, cols)
    report("3M ZGEMM %d^3 s=%d" % (n, s), got, nat, As, Bs)


@pytest.mark.parametrize("n", [8192, 16384])
@pytest.mark.parametrize("p", [2, 4])
def test_sgemm_reported(ctx, p, n):
    print("case SGEMM %d^3 p=%d" % (n, p), flush=True)
    A, B = real_pair(n, n, n, 9800 + p, dtype=torch.float32)
    C = ozk.ozk_sgemm(ctx, ozk.OZK_SCHEME1, p, A, B)
    rows, cols = sample(n, 20, p), sample(n, 20, p + 7)
    As, Bs = sub(A, B, rows, cols)
    assert np.array_equal(block(C, rows, cols), oracle.s1_sgemm(As, Bs, p))


def test_cgemm_4096(ctx):
    n, s = 4096, 8
    print("case CGEMM %d^3 s=%d" % (n, s), flush=True)
    A, B = complex_pair(n, n, n, 9900, dtype=torch.complex64)
    C = ozk.ozk_cgemm_3m(ctx, s, A, B)
    rows, cols = sample(n, 16, 3), sample(n, 16, 4)
    As, Bs = sub(A, B, rows, cols)
    assert np.array_equal(block(C, rows, cols), s2.z3m_cgemm(As, Bs, s))


@pytest.mark.parametrize("p", [4, 7])
def test_scheme1_configs_on_a_grid_of_whole_xcd_blocks(ctx, p):
    """1024 x 512 outputs: 32 or 64 workgroup tiles for every Scheme I tile
    variant, a multiple of the 8 XCDs, so raster 0 takes its XCD-aware order;
    every configuration equals the oracle."""
    M, N, K = 1024, 512, 256
    A = synth.phi_matrix(M, K, 1.0, 71 + p)
    B = synth.phi_matrix(K, N, 1.0, 72 + p)
    expect = oracle.s1_dgemm(A, B, p)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    for cfg in itertools.product(range(ozk.OZK_S1_VARIANTS), (0, 1), (1, 2, 4, 8), (1, 2)):
        ozk.ozk_config_set(ctx, ozk.OZK_OP_DGEMM, ozk.OZK_SCHEME1, p, M, N, K, cfg)
        got = ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME1, p, dA, dB)
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy(), expect), cfg


@pytest.mark.parametrize("cplx", [False, True])
def test_scheme2_configs_on_a_grid_of_whole_xcd_blocks(ctx, cplx):
    M, N, K, s = 1024, 512, 160, 9  # 8 to 64 tiles for every Scheme II tile
    if cplx:
        A = synth.complex_phi_matrix(M, K, 1.0, 81, 82)
        B = synth.complex_phi_matrix(K, N, 1.0, 83, 84)
        expect = s2.z3m_gemm(A, B, s)
        op = ozk.OZK_OP_ZGEMM
    else:
        A = synth.phi_matrix(M, K, 1.0, 81)
        B = synth.phi_matrix(K, N, 1.0, 83)
        expect = s2.s2_dgemm(A, B, s)
        op = ozk.OZK_OP_DGEMM
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    for v, raster, group in itertools.product(range(ozk.OZK_S2_VARIANTS), (0, 1), (1, 2, 8)):
        if cplx and v == ozk.OZK_S2_FUSED_CRT:
            continue
        ozk.ozk_config_set(ctx, op, ozk.OZK_SCHEME2, s, M, N, K, (v, raster, group, 1))
        got = ozk.ozk_zgemm_3m(ctx, s, dA, dB) if cplx else ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME2, s, dA, dB)
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy(), expect), (v, raster, group)
