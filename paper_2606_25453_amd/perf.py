"""Throughput of the library's paths on synthetic inputs (one JSON line each).

    python -m paper_2606_25453_amd.perf [--quick] [--out FILE]

Workloads (inputs resident in HBM, every kernel of the call timed with HIP
events on the launch stream, after untimed warm-up calls and tuning):
* Scheme I DGEMM, square n in {4096, 8192}, p in {6, 7, 8};
* Scheme I SGEMM (binary32 in and out), square n in {4096, 8192}, p in {2, 3, 4},
  against native float32 torch.matmul; Scheme II SGEMM (s = 8, 10) and 3M
  CGEMM (s = 8) at 4096^3 against native float32 / complex64;
* Scheme II DGEMM 4096^3 and 8192 x 8192 x 2048, s in {14, 16};
* Scheme II 3M ZGEMM 4096^3 and 8192^3, s = 16;
* Scheme I DGEMM fused against the unfused baseline (one GEMM per slice
  pair, INT32 planes through HBM), p = 7 at 4096^3 and 8192^3;
* Scheme II DGEMM (s = 14) and 3M ZGEMM (s = 16) fused against their
  unfused baselines (one GEMM per modular product, INT32 planes), 4096^3;
* Scheme I ZGEMM by 4M, p = 7, 4096^3 and 8192^3;
* Scheme II DGEMM with the CRT fused into the GEMM against the separate
  kernels, 4096^3 at s = 14 and 8192 x 8192 x 2048 at s = 16;
* a batch of 256 ZGEMMs with M, N, K log-uniform in [64, 1024], s = 16, one
  graph replay per call;
* the automatic path (selector decision on the device) at 4096^3 and 8192^3
  for a tolerance of 1e-13, against the fixed call at its decision.
With --sweep instead: the paper's size sweeps (Sec. V-B), Scheme I square n in
{1024, ..., 16384} with p in 3..8, Scheme II s in {8, ..., 16} at 4096^3 and
8192 x 8192 x 2048, 3M ZGEMM n in {2048, 4096, 8192}, and s = 15 at 16384^3
(real and complex), on inputs drawn on the device.
For each: emulated FP64 TFLOP/s (2MNK real, 8MNK complex per call), the INT8
operations of the GEMM step and their rate against the dense INT8 peak, and
the native float64 / complex128 torch.matmul on the same inputs.
"""
from __future__ import annotations

import argparse
import json
import math

import paper_2606_25453_amd as ozk

INT8_PEAK_TOPS = 5000.0


def _events(torch, n):
    return [torch.cuda.Event(enable_timing=True) for _ in range(n)]


def time_call(torch, fn, reps: int, warm: int = 2) -> float:
    """Mean ms of fn() over reps calls on the current stream."""
    for _ in range(warm):
        fn()
    a, b = _events(torch, 2)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    b.synchronize()
    return a.elapsed_time(b) / reps


def device_phi(torch, rows, cols, phi, seed, cplx=False):
    """(u - 0.5) exp(phi g) with u ~ U(0, 1), g ~ N(0, 1), drawn on the device
    (the recipe of the host generator, other random streams): the sweep's
    16384^2 inputs would take minutes on the host."""
    g = torch.Generator(device="cuda:0").manual_seed(seed)

    def part():
        u = torch.rand((rows, cols), generator=g, dtype=torch.float64, device="cuda:0")
        n = torch.randn((rows, cols), generator=g, dtype=torch.float64, device="cuda:0")
        return (u - 0.5) * torch.exp(phi * n)
    return torch.complex(part(), part()) if cplx else part()


def scheme1(torch, ctx, n, p, reps, inputs=None):
    import synth
    dev = "cuda:0"
    if inputs is None:
        A = torch.from_numpy(synth.phi_matrix(n, n, 1.0, synth.seed_for(2, n, 1.0, synth.ROLE_A))).to(dev)
        B = torch.from_numpy(synth.phi_matrix(n, n, 1.0, synth.seed_for(2, n, 1.0, synth.ROLE_B))).to(dev)
    else:
        A, B = inputs
    C = torch.empty((n, n), dtype=torch.float64, device=dev)
    _, cfg, gemm_ms = ozk.ozk_tune(ctx, ozk.OZK_OP_DGEMM, ozk.OZK_SCHEME1, p, A, B, C=C, reps=2)
    ws = torch.empty(ozk.ozk_workspace_size(ctx, ozk.OZK_OP_DGEMM, ozk.OZK_SCHEME1, n, n, n, p), dtype=torch.uint8,
                     device=dev)
    ms = time_call(torch, lambda: ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME1, p, A, B, C, ws=ws), reps)
    ms_nat = time_call(torch, lambda: torch.matmul(A, B, out=C), reps)
    ops = p * (p + 1) * n ** 3
    return {"path": "scheme1_dgemm", "M": n, "N": n, "K": n, "p": p, "config": cfg, "ms": round(ms, 4),
            "tflops": round(2.0 * n ** 3 / ms / 1e9, 3), "gemm_ms": round(gemm_ms, 4),
            "int8_ops": ops, "gemm_frac_int8_peak": round(ops / gemm_ms / 1e9 / INT8_PEAK_TOPS, 4),
            "native_tflops": round(2.0 * n ** 3 / ms_nat / 1e9, 3)}


def sgemm(torch, ctx, n, p, reps, inputs=None):
    """Scheme I SGEMM (binary32 in and out) against native float32
    torch.matmul (TF32 off).  The GEMM step is the DGEMM one, so its size
    class is tuned on the widened operands."""
    import synth
    dev = "cuda:0"
    if inputs is None:
        A = torch.from_numpy(synth.phi_matrix(n, n, 1.0, synth.seed_for(2, n, 1.0, synth.ROLE_A))).to(dev)
        B = torch.from_numpy(synth.phi_matrix(n, n, 1.0, synth.seed_for(2, n, 1.0, synth.ROLE_B))).to(dev)
    else:
        A, B = inputs
    A32, B32 = A.float(), B.float()
    A64, B64 = A32.double(), B32.double()
    _, cfg, gemm_ms = ozk.ozk_tune(ctx, ozk.OZK_OP_DGEMM, ozk.OZK_SCHEME1, p, A64, B64, reps=2)
    del A64, B64
    C = torch.empty((n, n), dtype=torch.float32, device=dev)
    ws = torch.empty(ozk.ozk_workspace_size(ctx, ozk.OZK_OP_DGEMM, ozk.OZK_SCHEME1, n, n, n, p), dtype=torch.uint8,
                     device=dev)
    ms = time_call(torch, lambda: ozk.ozk_sgemm(ctx, ozk.OZK_SCHEME1, p, A32, B32, C, ws=ws), reps)
    torch.backends.cuda.matmul.allow_tf32 = False
    ms_nat = time_call(torch, lambda: torch.matmul(A32, B32, out=C), reps)
    ops = p * (p + 1) * n ** 3
    return {"path": "scheme1_sgemm", "M": n, "N": n, "K": n, "p": p, "config": cfg, "ms": round(ms, 4),
            "tflops": round(2.0 * n ** 3 / ms / 1e9, 3), "gemm_ms": round(gemm_ms, 4),
            "int8_ops": ops, "gemm_frac_int8_peak": round(ops / gemm_ms / 1e9 / INT8_PEAK_TOPS, 4),
            "native_fp32_tflops": round(2.0 * n ** 3 / ms_nat / 1e9, 3)}


def unfused(torch, ctx, n, p, reps):
    """The fused Scheme I DGEMM against the unfused baseline (one GEMM per
    slice pair, INT32 planes through HBM; the paper's Eq. 9 against Eq. 10)."""
    A = device_phi(torch, n, n, 1.0, 91)
    B = device_phi(torch, n, n, 1.0, 92)
    C = torch.empty((n, n), dtype=torch.float64, device="cuda:0")
    _, cfg, gemm_ms = ozk.ozk_tune(ctx, ozk.OZK_OP_DGEMM, ozk.OZK_SCHEME1, p, A, B, C=C, reps=2)
    ws = torch.empty(ozk.ozk_workspace_size(ctx, ozk.OZK_OP_DGEMM, ozk.OZK_SCHEME1, n, n, n, p), dtype=torch.uint8,
                     device="cuda:0")
    ms_fused = time_call(torch, lambda: ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME1, p, A, B, C, ws=ws), reps)
    ref = C.clone()
    del ws
    wsu = torch.empty(ozk.ozk_s1_unfused_workspace_size(ctx, p, n, n, n), dtype=torch.uint8, device="cuda:0")
    ms_unf = time_call(torch, lambda: ozk.ozk_s1_dgemm_unfused(ctx, p, A, B, C, ws=wsu), reps)
    pairs = p * (p + 1) // 2
    return {"path": "scheme1_fused_vs_unfused", "M": n, "N": n, "K": n, "p": p, "ms_fused": round(ms_fused, 4),
            "tflops_fused": round(2.0 * n ** 3 / ms_fused / 1e9, 3), "ms_unfused": round(ms_unf, 4),
            "tflops_unfused": round(2.0 * n ** 3 / ms_unf / 1e9, 3), "bit_identical": bool(torch.equal(C, ref)),
            "model_bytes_fused": p * 2 * n * n + 8 * n * n,
            "model_bytes_unfused": pairs * 2 * n * n + 8 * pairs * n * n + 8 * n * n}


def embed4m(torch, A, B):
    """The real matrices whose product holds the 4M complex product (the
    layout ozk_zgemm uses for Scheme I): A viewed as M x 2K reals, and the
    2K x 2N matrix with rows 2k = (Re b, Im b), 2k+1 = (-Im b, Re b).  Used
    only to tune the GEMM step's size class on the embedded shape."""
    M, K = A.shape
    N = B.shape[1]
    A2 = torch.view_as_real(A).reshape(M, 2 * K)
    Br, Bi = B.real, B.imag
    B2 = torch.stack([torch.stack([Br, Bi], dim=2), torch.stack([-Bi, Br], dim=2)], dim=1).reshape(2 * K, 2 * N)
    return A2.contiguous(), B2.contiguous()


def zgemm4m(torch, ctx, n, p, reps):
    """Scheme I ZGEMM by 4M (4 p(p+1) MNK INT8 operations) against native
    complex128 torch.matmul and the Scheme II 3M call at s = 16."""
    A = device_phi(torch, n, n, 1.0, 61, True)
    B = device_phi(torch, n, n, 1.0, 62, True)
    A2, B2 = embed4m(torch, A, B)
    _, cfg, gemm_ms = ozk.ozk_tune(ctx, ozk.OZK_OP_DGEMM, ozk.OZK_SCHEME1, p, A2, B2, reps=2)
    del A2, B2
    torch.cuda.empty_cache()
    C = torch.empty((n, n), dtype=torch.complex128, device="cuda:0")
    ws = torch.empty(ozk.ozk_workspace_size(ctx, ozk.OZK_OP_ZGEMM, ozk.OZK_SCHEME1, n, n, n, p), dtype=torch.uint8,
                     device="cuda:0")
    ms = time_call(torch, lambda: ozk.ozk_zgemm(ctx, ozk.OZK_SCHEME1, p, A, B, C, ws=ws), reps)
    ms_nat = time_call(torch, lambda: torch.matmul(A, B, out=C), reps)
    flops = 8.0 * n ** 3
    ops = 4 * p * (p + 1) * n ** 3
    return {"path": "scheme1_zgemm_4m", "M": n, "N": n, "K": n, "p": p, "config": cfg, "ms": round(ms, 4),
            "tflops": round(flops / ms / 1e9, 3), "gemm_ms": round(gemm_ms, 4), "int8_ops": ops,
            "gemm_frac_int8_peak": round(ops / gemm_ms / 1e9 / INT8_PEAK_TOPS, 4),
            "native_tflops": round(flops / ms_nat / 1e9, 3)}


def s2_unfused(torch, ctx, n, s, cplx, reps):
    """The fused Scheme II (or 3M) call against the unfused baseline (INT32
    planes through HBM; the paper's Eq. 14 against Eq. 15, Eq. 17 against
    Eq. 18)."""
    A = device_phi(torch, n, n, 1.0, 51, cplx)
    B = device_phi(torch, n, n, 1.0, 52, cplx)
    op = ozk.OZK_OP_ZGEMM if cplx else ozk.OZK_OP_DGEMM
    C = torch.empty((n, n), dtype=A.dtype, device="cuda:0")
    _, cfg, _ = ozk.ozk_tune(ctx, op, ozk.OZK_SCHEME2, s, A, B, C=C, reps=2)
    ws = torch.empty(ozk.ozk_workspace_size(ctx, op, ozk.OZK_SCHEME2, n, n, n, s), dtype=torch.uint8, device="cuda:0")
    if cplx:
        ms_fused = time_call(torch, lambda: ozk.ozk_zgemm_3m(ctx, s, A, B, C, ws=ws), reps)
    else:
        ms_fused = time_call(torch, lambda: ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME2, s, A, B, C, ws=ws), reps)
    ref = C.clone()
    del ws
    wsu = torch.empty(ozk.ozk_s2_unfused_workspace_size(ctx, s, int(cplx), n, n, n), dtype=torch.uint8,
                      device="cuda:0")
    ms_unf = time_call(torch, lambda: ozk.ozk_s2_gemm_unfused(ctx, s, A, B, C, ws=wsu), reps)
    q = 3 if cplx else 1
    flops = (8.0 if cplx else 2.0) * n ** 3
    return {"path": "scheme2_3m_fused_vs_unfused" if cplx else "scheme2_fused_vs_unfused", "M": n, "N": n, "K": n,
            "s": s, "ms_fused": round(ms_fused, 4), "tflops_fused": round(flops / ms_fused / 1e9, 3),
            "ms_unfused": round(ms_unf, 4), "tflops_unfused": round(flops / ms_unf / 1e9, 3),
            "bit_identical": bool(torch.equal(C, ref)),
            "model_bytes_fused": s * (q * 2 * n * n + (2 if cplx else 1) * n * n),
            "model_bytes_unfused": s * (q * 2 * n * n + 8 * q * n * n + (2 if cplx else 1) * n * n)}


def scheme2_f32(torch, ctx, n, s, cplx, reps):
    """Scheme II SGEMM or 3M CGEMM (binary32 in and out) against native
    float32 / complex64 torch.matmul (TF32 off); the GEMM step is tuned on
    the widened operands."""
    A = device_phi(torch, n, n, 1.0, 81, cplx)
    B = device_phi(torch, n, n, 1.0, 82, cplx)
    op = ozk.OZK_OP_ZGEMM if cplx else ozk.OZK_OP_DGEMM
    _, cfg, gemm_ms = ozk.ozk_tune(ctx, op, ozk.OZK_SCHEME2, s, A, B, reps=2)
    A32 = A.to(torch.complex64 if cplx else torch.float32)
    B32 = B.to(torch.complex64 if cplx else torch.float32)
    del A, B
    C = torch.empty((n, n), dtype=A32.dtype, device="cuda:0")
    ws = torch.empty(ozk.ozk_workspace_size(ctx, op, ozk.OZK_SCHEME2, n, n, n, s), dtype=torch.uint8, device="cuda:0")
    if cplx:
        ms = time_call(torch, lambda: ozk.ozk_cgemm_3m(ctx, s, A32, B32, C, ws=ws), reps)
    else:
        ms = time_call(torch, lambda: ozk.ozk_sgemm(ctx, ozk.OZK_SCHEME2, s, A32, B32, C, ws=ws), reps)
    torch.backends.cuda.matmul.allow_tf32 = False
    ms_nat = time_call(torch, lambda: torch.matmul(A32, B32, out=C), reps)
    flops = (8.0 if cplx else 2.0) * n ** 3
    ops = (6 if cplx else 2) * s * n ** 3
    return {"path": "scheme2_cgemm_3m" if cplx else "scheme2_sgemm", "M": n, "N": n, "K": n, "s": s, "config": cfg,
            "ms": round(ms, 4), "tflops": round(flops / ms / 1e9, 3), "gemm_ms": round(gemm_ms, 4),
            "int8_ops": ops, "gemm_frac_int8_peak": round(ops / gemm_ms / 1e9 / INT8_PEAK_TOPS, 4),
            "native_tflops": round(flops / ms_nat / 1e9, 3)}


def scheme2(torch, ctx, M, N, K, s, cplx, reps, inputs=None):
    import synth
    dev = "cuda:0"
    if inputs is not None:
        A, B = inputs
        op, dt = (ozk.OZK_OP_ZGEMM, torch.complex128) if cplx else (ozk.OZK_OP_DGEMM, torch.float64)
    elif cplx:
        A = torch.from_numpy(synth.complex_phi_matrix(M, K, 1.0, 31, 32)).to(dev)
        B = torch.from_numpy(synth.complex_phi_matrix(K, N, 1.0, 33, 34)).to(dev)
        op, dt = ozk.OZK_OP_ZGEMM, torch.complex128
    else:
        A = torch.from_numpy(synth.phi_matrix(M, K, 1.0, 31)).to(dev)
        B = torch.from_numpy(synth.phi_matrix(K, N, 1.0, 33)).to(dev)
        op, dt = ozk.OZK_OP_DGEMM, torch.float64
    C = torch.empty((M, N), dtype=dt, device=dev)
    _, cfg, gemm_ms = ozk.ozk_tune(ctx, op, ozk.OZK_SCHEME2, s, A, B, C=C, reps=2)
    ws = torch.empty(ozk.ozk_workspace_size(ctx, op, ozk.OZK_SCHEME2, M, N, K, s), dtype=torch.uint8, device=dev)
    if cplx:
        ms = time_call(torch, lambda: ozk.ozk_zgemm_3m(ctx, s, A, B, C, ws=ws), reps)
    else:
        ms = time_call(torch, lambda: ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME2, s, A, B, C, ws=ws), reps)
    ms_nat = time_call(torch, lambda: torch.matmul(A, B, out=C), reps)
    flops = (8.0 if cplx else 2.0) * M * N * K
    ops = (6 if cplx else 2) * s * M * N * K
    return {"path": "scheme2_zgemm_3m" if cplx else "scheme2_dgemm", "M": M, "N": N, "K": K, "s": s,
            "config": cfg, "ms": round(ms, 4), "tflops": round(flops / ms / 1e9, 3), "gemm_ms": round(gemm_ms, 4),
            "int8_ops": ops, "gemm_frac_int8_peak": round(ops / gemm_ms / 1e9 / INT8_PEAK_TOPS, 4),
            "native_tflops": round(flops / ms_nat / 1e9, 3)}


def fused_crt(torch, ctx, M, N, K, s, reps):
    """Scheme II DGEMM with the CRT fused into the GEMM (variant
    OZK_S2_FUSED_CRT) against the separate kernels at the tuned variant."""
    import synth
    dev = "cuda:0"
    A = torch.from_numpy(synth.phi_matrix(M, K, 1.0, 31)).to(dev)
    B = torch.from_numpy(synth.phi_matrix(K, N, 1.0, 33)).to(dev)
    C = torch.empty((M, N), dtype=torch.float64, device=dev)
    _, cfg, _ = ozk.ozk_tune(ctx, ozk.OZK_OP_DGEMM, ozk.OZK_SCHEME2, s, A, B, C=C, reps=2)
    ws = torch.empty(ozk.ozk_workspace_size(ctx, ozk.OZK_OP_DGEMM, ozk.OZK_SCHEME2, M, N, K, s), dtype=torch.uint8,
                     device=dev)
    ms_sep = time_call(torch, lambda: ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME2, s, A, B, C, ws=ws), reps)
    sep = C.clone()
    ozk.ozk_config_set(ctx, ozk.OZK_OP_DGEMM, ozk.OZK_SCHEME2, s, M, N, K, (ozk.OZK_S2_FUSED_CRT, 0, 4, 1))
    ms_fused = time_call(torch, lambda: ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME2, s, A, B, C, ws=ws), reps)
    same = bool(torch.equal(C, sep))
    ozk.ozk_config_set(ctx, ozk.OZK_OP_DGEMM, ozk.OZK_SCHEME2, s, M, N, K, cfg)
    flops = 2.0 * M * N * K
    return {"path": "scheme2_dgemm_fused_crt", "M": M, "N": N, "K": K, "s": s, "ms_fused": round(ms_fused, 4),
            "tflops_fused": round(flops / ms_fused / 1e9, 3), "ms_separate": round(ms_sep, 4),
            "tflops_separate": round(flops / ms_sep / 1e9, 3), "separate_config": cfg, "bit_identical": same}


def batch(torch, ctx, count, s, reps):
    import synth
    dev = "cuda:0"
    dims = synth.log_uniform_ints(3 * count, 64, 1024, synth.seed_for(4, count, 1.0, 0)).reshape(count, 3)
    g = torch.Generator(device="cpu").manual_seed(4)
    dA, dB, dC = [], [], []
    flops = ops = 0
    for (M, N, K) in dims:
        M, N, K = int(M), int(N), int(K)
        a = (torch.rand((M, K), generator=g, dtype=torch.float64) - 0.5) + 1j * (
            torch.rand((M, K), generator=g, dtype=torch.float64) - 0.5)
        b = (torch.rand((K, N), generator=g, dtype=torch.float64) - 0.5) + 1j * (
            torch.rand((K, N), generator=g, dtype=torch.float64) - 0.5)
        dA.append(a.to(dev))
        dB.append(b.to(dev))
        dC.append(torch.empty((M, N), dtype=torch.complex128, device=dev))
        flops += 8.0 * M * N * K
        ops += 6 * s * M * N * K
    plan = ozk.BatchPlan(ctx, ozk.OZK_OP_ZGEMM, ozk.OZK_SCHEME2, s, list(zip(dA, dB, dC)))
    default_tiles = plan.tiles()
    ms_default = time_call(torch, plan.run, reps)
    plan.tune(reps=3)  # the tile of each size class, on these problems
    tiles = plan.tiles()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        plan.run(stream=side)
        torch.cuda.synchronize()
        with torch.cuda.graph(graph, stream=side):
            plan.run(stream=side)
    torch.cuda.current_stream().wait_stream(side)
    ms_graph = time_call(torch, graph.replay, reps)
    ms_eager = time_call(torch, plan.run, reps)
    plan.close()
    return {"path": "batch_zgemm_3m", "count": count, "s": s, "ms_graph": round(ms_graph, 4),
            "ms_eager": round(ms_eager, 4), "tflops": round(flops / ms_graph / 1e9, 3), "int8_ops": ops,
            "end_to_end_frac_int8_peak": round(ops / ms_graph / 1e9 / INT8_PEAK_TOPS, 4),
            "large_tile_problems": sum(tiles), "ms_eager_untuned": round(ms_default, 4),
            "large_tile_problems_untuned": sum(default_tiles)}


def auto(torch, ctx, n, tol, reps):
    """ozk_dgemm_auto (decision on the device, both pipelines enqueued, the
    one not chosen returning at once) against ozk_dgemm at the decision."""
    import synth
    dev = "cuda:0"
    A = torch.from_numpy(synth.phi_matrix(n, n, 1.0, synth.seed_for(2, n, 1.0, synth.ROLE_A))).to(dev)
    B = torch.from_numpy(synth.phi_matrix(n, n, 1.0, synth.seed_for(2, n, 1.0, synth.ROLE_B))).to(dev)
    C = torch.empty((n, n), dtype=torch.float64, device=dev)
    info = torch.empty(ozk.OZK_SELECTOR_INFO, dtype=torch.int32, device=dev)
    ws = torch.empty(ozk.ozk_workspace_size(ctx, ozk.OZK_OP_DGEMM, ozk.OZK_SCHEME1, n, n, n, 0), dtype=torch.uint8,
                     device=dev)
    ozk.ozk_dgemm_auto(ctx, tol, A, B, C, ws=ws, info=info)
    torch.cuda.synchronize()
    d = [int(x) for x in info.cpu()]
    scheme, ps = (ozk.OZK_SCHEME1, d[0]) if d[4] == 1 else (ozk.OZK_SCHEME2, d[5])
    ozk.ozk_tune(ctx, ozk.OZK_OP_DGEMM, scheme, ps, A, B, C=C, reps=2)
    ms_auto = time_call(torch, lambda: ozk.ozk_dgemm_auto(ctx, tol, A, B, C, ws=ws, info=info), reps)
    wsf = torch.empty(ozk.ozk_workspace_size(ctx, ozk.OZK_OP_DGEMM, scheme, n, n, n, ps), dtype=torch.uint8,
                      device=dev)
    ms_fixed = time_call(torch, lambda: ozk.ozk_dgemm(ctx, scheme, ps, A, B, C, ws=wsf), reps)
    return {"path": "dgemm_auto", "M": n, "N": n, "K": n, "tol": tol,
            "decision": {"scheme": "I" if scheme == ozk.OZK_SCHEME1 else "II", "p_or_s": ps, "p_net": d[1],
                         "p_bound": d[2]},
            "ms": round(ms_auto, 4), "tflops": round(2.0 * n ** 3 / ms_auto / 1e9, 3),
            "ms_fixed_at_decision": round(ms_fixed, 4), "overhead_pct": round(100.0 * (ms_auto / ms_fixed - 1), 2)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--quick", action="store_true", help="the smaller sizes only")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--out", default=None, help="also append the lines to this file")
    ap.add_argument("--only", default=None,
                    help="comma-separated subset of s1, sgemm, unfused, s2, s2f32, fused, s2unf, z4m, batch, auto")
    ap.add_argument("--sweep", action="store_true", help="the size sweeps instead of the default workloads")
    args = ap.parse_args()
    import torch
    ozk.library()
    ctx = ozk.Context(0)
    if args.sweep:
        sweep(torch, ctx, args)
        ctx.close()
        return
    try:
        actx = ozk.Context(0, selector="default")
        net = True
    except ValueError:  # shipped parameters of another network shape: the bounds decide
        actx = ozk.Context(0)
        net = False
    jobs = [("s1", 4096, p) for p in (6, 7, 8)]
    jobs += [("s2", 4096, 4096, 4096, s, False) for s in (14, 16)]
    jobs += [("s2", 8192, 8192, 2048, s, False) for s in (14, 16)]
    jobs += [("s2", 4096, 4096, 4096, 16, True)]
    jobs += [("fused", 4096, 4096, 4096, 14), ("fused", 8192, 8192, 2048, 16)]
    jobs += [("sgemm", 4096, p) for p in (2, 3, 4)]
    jobs += [("s2f32", 4096, s, False) for s in (8, 10)] + [("s2f32", 4096, 8, True)]
    jobs += [("unfused", 4096, 7)]
    jobs += [("s2unf", 4096, 14, False), ("s2unf", 4096, 16, True)]
    jobs += [("z4m", 4096, 7)]
    jobs += [("batch", 256, 16)]
    jobs += [("auto", 4096, 1e-13)]
    if not args.quick:
        jobs += [("auto", 8192, 1e-13), ("auto", 8192, 1e-10)]
        jobs += [("s1", 8192, p) for p in (6, 7, 8)]
        jobs += [("sgemm", 8192, p) for p in (2, 3, 4)]
        jobs += [("unfused", 8192, 7)]
        jobs += [("s2", 8192, 8192, 8192, 16, True)]
        jobs += [("z4m", 8192, 7)]
    if args.only:
        keep = set(args.only.split(","))
        jobs = [j for j in jobs if j[0] in keep]
    out = open(args.out, "a") if args.out else None
    for job in jobs:
        if job[0] == "s1":
            r = scheme1(torch, ctx, job[1], job[2], args.reps)
        elif job[0] == "s2":
            r = scheme2(torch, ctx, job[1], job[2], job[3], job[4], job[5], args.reps)
        elif job[0] == "auto":
            r = auto(torch, actx, job[1], job[2], args.reps)
            r["network"] = net
        elif job[0] == "fused":
            r = fused_crt(torch, ctx, job[1], job[2], job[3], job[4], args.reps)
        elif job[0] == "sgemm":
            r = sgemm(torch, ctx, job[1], job[2], args.reps)
        elif job[0] == "unfused":
            r = unfused(torch, ctx, job[1], job[2], args.reps)
        elif job[0] == "s2f32":
            r = scheme2_f32(torch, ctx, job[1], job[2], job[3], args.reps)
        elif job[0] == "z4m":
            r = zgemm4m(torch, ctx, job[1], job[2], args.reps)
        elif job[0] == "s2unf":
            r = s2_unfused(torch, ctx, job[1], job[2], job[3], args.reps)
        else:
            r = batch(torch, ctx, job[1], job[2], args.reps)
        line = json.dumps(r)
        print(line, flush=True)
        if out:
            out.write(line + "\n")
            out.flush()
        torch.cuda.empty_cache()
    ctx.close()
    actx.close()


def sweep(torch, ctx, args):
    out = open(args.out, "a") if args.out else None
    jobs = [("s1", n, p) for n in (1024, 2048, 4096, 8192, 16384) for p in range(3, 9)]
    jobs += [("s2", 4096, 4096, 4096, s, False) for s in (8, 10, 12, 14, 16)]
    jobs += [("s2", 8192, 8192, 2048, s, False) for s in (8, 10, 12, 14, 16)]
    jobs += [("s2", n, n, n, 16, True) for n in (2048, 4096, 8192)]
    jobs += [("s2", 16384, 16384, 16384, 15, False), ("s2", 16384, 16384, 16384, 15, True)]
    jobs += [("sgemm", n, p) for n in (4096, 8192, 16384) for p in (1, 2, 3, 4)]
    if args.only:
        keep = set(args.only.split(","))
        jobs = [j for j in jobs if j[0] in keep]
    key, inputs = None, None
    for job in jobs:
        shape = (job[1], job[1], job[1], False) if job[0] in ("s1", "sgemm") else job[1:4] + (job[5],)
        if shape != key:
            inputs = None
            torch.cuda.empty_cache()
            M, N, K, cplx = shape
            inputs = (device_phi(torch, M, K, 1.0, 71, cplx), device_phi(torch, K, N, 1.0, 72, cplx))
            key = shape
        if job[0] == "s1":
            r = scheme1(torch, ctx, job[1], job[2], args.reps, inputs)
        elif job[0] == "sgemm":
            r = sgemm(torch, ctx, job[1], job[2], args.reps, inputs)
        else:
            r = scheme2(torch, ctx, job[1], job[2], job[3], job[4], job[5], args.reps, inputs)
        r["inputs"] = "device phi = 1"
        line = json.dumps(r)
        print(line, flush=True)
        if out:
            out.write(line + "\n")
            out.flush()


if __name__ == "__main__":
    main()
