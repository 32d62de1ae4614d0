"""Training and loading of the learned slice / modulus count selector.

Everything numeric runs on the GPU through the library's C ABI:
* problems: synthetic (u - 0.5) exp(phi g) matrices with phi ~ U(0, 4) for A
  and B independently, M, N log-uniform in [256, 4096] and K log-uniform in
  [256, 16384] (the paper's generator, Sec. V-B, Eq. 19, with random
  conditioning; K reaches the 16384 the selector is trusted up to);
* labels: the componentwise error of the emulated product against the
  double-double reference kernel, E_cw = max |C - C_dd| / (|A||B|), for
  Scheme I with p = 1..8 and Scheme II with s = 1..20, and for each of four
  tolerances drawn log-uniformly in [1e-16, 1e-5] the smallest p (9 if none)
  and the smallest s (21 if none) whose error is at most half the
  tolerance (the training targets), and the smallest counts whose error is
  at most the tolerance itself (the calibration targets).  The error is
  measured on up to 512 x 512 outputs (rows and columns drawn at random; all
  of them for smaller products): the row (column) scales of both schemes
  depend only on that row of A (column of B), so the emulation of the
  sampled rows times the sampled columns gives exactly the full product's
  values there, and the factor of two of the training targets covers the
  outputs not sampled;
* features: the selector's own exponent-statistics kernels on the full A, B;
* training: the library's MLP forward / gradient / Adam kernels on the
  ordinal binary cross-entropy of the 28 heads;
* calibration on held-out problems: per head the largest threshold below
  which no held-out sample whose error at that count exceeds the tolerance
  falls (so no held-out sample gets a result outside its tolerance), lowered
  by half a logit for the problems not seen.
PyTorch only allocates and fills device memory and does the small
element-wise bookkeeping around those calls.

    python -m paper_2606_25453_amd.selector --train 20000 --val 2000

The trained parameters ship as selector_weights.json next to this file.
"""
from __future__ import annotations

import json
import math
import os
from typing import Dict, List, Tuple

import paper_2606_25453_amd as ozk

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "selector_weights.json")
P_HEADS, S_HEADS = 8, 20
N_HEADS = P_HEADS + S_HEADS
SAMPLE = 512          # rows and columns of the sampled outputs per problem
LABEL_MARGIN = 0.5    # a label's error must be at most this fraction of the tolerance


def _torch():
    import torch
    return torch


def random_problem(gen, M: int, N: int, K: int, phi_a: float, phi_b: float, device):
    torch = _torch()
    a = (torch.rand((M, K), generator=gen, device=device, dtype=torch.float64) - 0.5) * torch.exp(
        phi_a * torch.randn((M, K), generator=gen, device=device, dtype=torch.float64))
    b = (torch.rand((K, N), generator=gen, device=device, dtype=torch.float64) - 0.5) * torch.exp(
        phi_b * torch.randn((K, N), generator=gen, device=device, dtype=torch.float64))
    return a, b


def dd_reference(ctx, A, B, rows=None, cols=None):
    """(hi, lo, absab) for all outputs, or for the listed ones."""
    torch = _torch()
    M, K = A.shape
    N = B.shape[1]
    if rows is None:
        ii, jj = torch.meshgrid(torch.arange(M, device=A.device), torch.arange(N, device=A.device), indexing="ij")
        rows, cols = ii.reshape(-1).contiguous(), jj.reshape(-1).contiguous()
    n = rows.numel()
    hi = torch.empty(n, dtype=torch.float64, device=A.device)
    lo = torch.empty_like(hi)
    ab = torch.empty_like(hi)
    st = ozk.library().ozk_ref_dd(ctx.handle, M, N, K, A.data_ptr(), ozk._ld(A), B.data_ptr(), ozk._ld(B), n,
                                  rows.data_ptr(), cols.data_ptr(), hi.data_ptr(), lo.data_ptr(), ab.data_ptr(),
                                  ozk._stream(None))
    ozk._check("ozk_ref_dd", st, ctx)
    return hi, lo, ab


def e_cw_dev(C, hi, lo, ab):
    """max |C - hi - lo| / (|A||B|) over entries with a nonzero scale, as a
    device scalar."""
    torch = _torch()
    err = ((C.reshape(-1) - hi) - lo).abs()
    ok = (ab > 0) & torch.isfinite(err)
    return torch.where(ok, err / torch.where(ok, ab, torch.ones_like(ab)), torch.zeros_like(err)).max()


def e_cw(C, hi, lo, ab) -> float:
    return float(e_cw_dev(C, hi, lo, ab))


def sampled_rows_cols(gen, M: int, N: int, device):
    torch = _torch()
    rows = torch.randperm(M, generator=gen, device=device)[:SAMPLE].sort().values if M > SAMPLE else \
        torch.arange(M, device=device)
    cols = torch.randperm(N, generator=gen, device=device)[:SAMPLE].sort().values if N > SAMPLE else \
        torch.arange(N, device=device)
    return rows, cols


def error_curves(ctx, A, B, rows, cols):
    """E_cw of Scheme I for p = 1..8 and of Scheme II for s = 1..20 on the
    outputs at (rows x cols): the emulation of the sampled sub-problem."""
    torch = _torch()
    As = A.index_select(0, rows).contiguous()
    Bs = B.index_select(1, cols).contiguous()
    hi, lo, ab = dd_reference(ctx, As, Bs)
    errs = [e_cw_dev(ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME1, p, As, Bs), hi, lo, ab) for p in range(1, P_HEADS + 1)]
    errs += [e_cw_dev(ozk.ozk_dgemm(ctx, ozk.OZK_SCHEME2, s, As, Bs), hi, lo, ab) for s in range(1, S_HEADS + 1)]
    out = torch.stack(errs).cpu().tolist()
    return out[:P_HEADS], out[P_HEADS:]


def label_from_curve(curve: List[float], tol: float, margin: float = LABEL_MARGIN) -> int:
    """The smallest count whose error is at most margin * tol (len + 1 if none)."""
    for c, err in enumerate(curve, start=1):
        if err <= margin * tol:
            return c
    return len(curve) + 1


def features(ctx, A, B, tol: float):
    """(34 features, info[8], counters) from the selector's own device kernels."""
    torch = _torch()
    M, K = A.shape
    N = B.shape[1]
    dev = A.device
    e = torch.empty(max(M, 1), dtype=torch.int32, device=dev)
    f = torch.empty(max(N, 1), dtype=torch.int32, device=dev)
    cnt = torch.empty(34, dtype=torch.int32, device=dev)
    info = torch.empty(ozk.OZK_SELECTOR_INFO, dtype=torch.int32, device=dev)
    feat = torch.empty(34, dtype=torch.float32, device=dev)
    st = ozk.library().ozk_select(ctx.handle, float(tol), M, N, K, A.data_ptr(), ozk._ld(A), B.data_ptr(), ozk._ld(B),
                                  e.data_ptr(), f.data_ptr(), cnt.data_ptr(), info.data_ptr(), feat.data_ptr(),
                                  ozk._stream(None))
    ozk._check("ozk_select", st, ctx)
    return feat, info, cnt


def _log_uniform(u: float, lo: int, hi: int) -> int:
    return min(hi, int(math.exp(math.log(lo) + (math.log(hi + 1) - math.log(lo)) * u)))


def build_dataset(ctx, count: int, seed: int, mn=(256, 4096), k_range=(256, 16384), tols_per_problem: int = 4,
                  device="cuda:0"):
    """Features (n x 34), Scheme I labels p (n), Scheme II labels s (n), the
    a-priori bounds' decisions (n x 2), the per-problem error curves and the
    labels at the full tolerance (n x 2: p, s)."""
    torch = _torch()
    host_gen = torch.Generator().manual_seed(seed)
    gen = torch.Generator(device=device).manual_seed(seed)
    X, lp, ls, bounds, curves, full = [], [], [], [], [], []
    for i in range(count):
        if i % 500 == 0:
            print("dataset seed %d: problem %d of %d" % (seed, i, count), flush=True)
        u = torch.rand(3 + 2 + tols_per_problem, generator=host_gen, dtype=torch.float64).tolist()
        M, N = _log_uniform(u[0], *mn), _log_uniform(u[1], *mn)
        K = _log_uniform(u[2], *k_range)
        phi_a, phi_b = 4.0 * u[3], 4.0 * u[4]
        A, B = random_problem(gen, M, N, K, phi_a, phi_b, device)
        rows, cols = sampled_rows_cols(gen, M, N, device)
        cp, cs = error_curves(ctx, A, B, rows, cols)
        curves.append({"M": M, "N": N, "K": K, "phi_a": phi_a, "phi_b": phi_b, "p": cp, "s": cs})
        for v in u[5:]:
            tol = 10.0 ** (-16.0 + 11.0 * v)
            feat, info, _ = features(ctx, A, B, tol)
            X.append(feat.clone())
            lp.append(label_from_curve(cp, tol))
            ls.append(label_from_curve(cs, tol))
            full.append((label_from_curve(cp, tol, 1.0), label_from_curve(cs, tol, 1.0)))
            bounds.append(info[[2, 6]].clone())
        del A, B
    return (torch.stack(X), torch.tensor(lp, dtype=torch.int64), torch.tensor(ls, dtype=torch.int64),
            torch.stack(bounds).cpu(), curves, torch.tensor(full, dtype=torch.int64))


def ordinal_targets(lp, ls):
    """y[:, t-1] = (p > t) for t = 1..8, y[:, 7+t] = (s > t) for t = 1..20."""
    torch = _torch()
    tp = torch.arange(1, P_HEADS + 1, device=lp.device).reshape(1, -1)
    ts = torch.arange(1, S_HEADS + 1, device=ls.device).reshape(1, -1)
    return torch.cat([(lp.reshape(-1, 1) > tp), (ls.reshape(-1, 1) > ts)], dim=1).to(torch.float32)


def init_params(seed: int, device):
    torch = _torch()
    g = torch.Generator(device="cpu").manual_seed(seed)
    shapes = [(34, 64), (64,), (64, 64), (64,), (64, N_HEADS), (N_HEADS,)]
    parts = []
    for sh in shapes:
        if len(sh) == 2:
            parts.append((torch.randn(sh, generator=g) * math.sqrt(2.0 / sh[0])).reshape(-1))
        else:
            parts.append(torch.zeros(sh))
    w = torch.cat(parts).to(torch.float32).to(device).contiguous()
    assert w.numel() == ozk.OZK_SELECTOR_PARAMS
    return w


def train(ctx, X, Y, steps: int = 6000, batch: int = 512, lr: float = 3e-3, seed: int = 0):
    """Mini-batch Adam on the ordinal cross-entropy with the library kernels
    (learning rate divided by 10 for the last quarter of the steps)."""
    torch = _torch()
    dev = X.device
    w = init_params(seed, dev)
    m = torch.zeros_like(w)
    v = torch.zeros_like(w)
    g = torch.empty_like(w)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    gen = torch.Generator(device=dev).manual_seed(seed + 1)
    lib = ozk.library()
    st_ = ozk._stream(None)
    hist = []
    n = X.shape[0]
    for step in range(1, steps + 1):
        idx = torch.randint(0, n, (min(batch, n),), generator=gen, device=dev)
        xb = X[idx].contiguous()
        yb = Y[idx].contiguous()
        st = lib.ozk_mlp_grad(ctx.handle, w.data_ptr(), xb.data_ptr(), yb.data_ptr(), xb.shape[0], g.data_ptr(),
                              loss.data_ptr(), st_)
        ozk._check("ozk_mlp_grad", st, ctx)
        rate = lr if step <= 3 * steps // 4 else lr / 10
        st = lib.ozk_mlp_adam(ctx.handle, w.data_ptr(), g.data_ptr(), m.data_ptr(), v.data_ptr(), step, rate, st_)
        ozk._check("ozk_mlp_adam", st, ctx)
        if step % 100 == 0:
            hist.append(float(loss))
        if step % 1000 == 0:
            print("training step %d: loss %.5f" % (step, hist[-1]), flush=True)
    return w, hist


def forward(ctx, w, X):
    torch = _torch()
    out = torch.empty((X.shape[0], N_HEADS), dtype=torch.float32, device=X.device)
    st = ozk.library().ozk_mlp_forward(ctx.handle, w.data_ptr(), X.contiguous().data_ptr(), X.shape[0],
                                       out.data_ptr(), ozk._stream(None))
    ozk._check("ozk_mlp_forward", st, ctx)
    return out


def counts(logits, thresholds, margin: int = 0):
    """(p_net, s_net) of the decision rule for per-head thresholds."""
    torch = _torch()
    up = torch.sigmoid(logits) > thresholds.reshape(1, -1).to(logits.device)
    p = torch.clamp(1 + up[:, :P_HEADS].sum(dim=1) + margin, max=9)
    s = torch.clamp(1 + up[:, P_HEADS:].sum(dim=1) + margin, max=21)
    return p, s


def calibrate(ctx, w, X, Y, slack: float = 0.5):
    """Per-head thresholds: sigmoid(min logit over the held-out samples that
    need the head on - slack), so that every such sample turns it on with
    room to spare; 0.5 for a head no held-out sample needs.  Y holds the
    targets at the full tolerance: a sample needs head t when its error at
    count t exceeds the tolerance."""
    torch = _torch()
    logits = forward(ctx, w, X)
    thr = torch.full((N_HEADS,), 0.5, dtype=torch.float32)
    for h in range(N_HEADS):
        pos = Y[:, h] > 0.5
        if bool(pos.any()):
            z = float(logits[pos, h].min()) - slack
            thr[h] = min(0.5, max(1e-6, 1.0 / (1.0 + math.exp(-z))))
    return thr


def decisions(p_net, s_net, bounds):
    """(scheme-I count used or 9, Scheme II count used or 0) of the rule
    p = min(p_net, p_bound); Scheme II at min(s_net, s_bound) when p = 9."""
    torch = _torch()
    pb, sb = bounds[:, 0].to(p_net.device), bounds[:, 1].to(p_net.device)
    p = torch.minimum(p_net, pb)
    s = torch.where(p > 8, torch.clamp(torch.minimum(s_net, sb), max=20), torch.zeros_like(p))
    return p, s


def save(path: str, w, thresholds, margin: int, meta: Dict) -> None:
    with open(path, "w") as fh:
        json.dump({"params": [float(x) for x in w.cpu().tolist()],
                   "thresholds": [float(x) for x in thresholds.tolist()], "margin": margin, "meta": meta}, fh)


def load(path: str = WEIGHTS):
    with open(path) as fh:
        return json.load(fh)


def install(ctx, path: str = WEIGHTS) -> Dict:
    """Load the shipped (or given) parameters into the context."""
    import ctypes
    d = load(path)
    if len(d["params"]) != ozk.OZK_SELECTOR_PARAMS or len(d.get("thresholds", ())) != ozk.OZK_SELECTOR_HEADS:
        raise ValueError("%s holds parameters of another network shape" % path)
    arr = (ctypes.c_float * len(d["params"]))(*d["params"])
    thr = (ctypes.c_float * ozk.OZK_SELECTOR_HEADS)(*d["thresholds"])
    st = ozk.library().ozk_selector_load(ctx.handle, ctypes.cast(arr, ctypes.c_void_p), len(d["params"]),
                                         ctypes.cast(thr, ctypes.c_void_p), int(d["margin"]))
    ozk._check("ozk_selector_load", st, ctx)
    return d


def main():
    import argparse
    import time
    torch = _torch()
    ap = argparse.ArgumentParser(description="train the slice / modulus count selector on the GPU")
    ap.add_argument("--train", type=int, default=20000)
    ap.add_argument("--val", type=int, default=2000)
    ap.add_argument("--steps", type=int, default=8000)
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--data", default=None, help="also save the datasets (torch.save) here")
    a = ap.parse_args()
    ctx = ozk.Context(0)
    t0 = time.time()
    Xtr, ptr, str_, btr, ctr, ftr = build_dataset(ctx, a.train, seed=1)
    Xva, pva, sva, bva, cva, fva = build_dataset(ctx, a.val, seed=2)
    t_data = time.time() - t0
    print("datasets %.1fs: train %d val %d samples" % (t_data, len(ptr), len(pva)), flush=True)
    if a.data:
        torch.save({"Xtr": Xtr.cpu(), "ptr": ptr, "str": str_, "btr": btr, "ftr": ftr, "Xva": Xva.cpu(), "pva": pva,
                    "sva": sva, "bva": bva, "fva": fva}, a.data)
    dev = Xtr.device
    Ytr = ordinal_targets(ptr.to(dev), str_.to(dev))
    Yva = ordinal_targets(pva.to(dev), sva.to(dev))
    w, hist = train(ctx, Xtr, Ytr, steps=a.steps)
    thr = calibrate(ctx, w, Xva, ordinal_targets(fva[:, 0].to(dev), fva[:, 1].to(dev)))
    p_net, s_net = counts(forward(ctx, w, Xva), thr)
    p_use, s_use = decisions(p_net, s_net, bva)
    pva_d, sva_d = pva.to(dev), sva.to(dev)
    pf, sf = fva[:, 0].to(dev), fva[:, 1].to(dev)
    pb, sb = bva[:, 0].to(dev), bva[:, 1].to(dev)
    to2 = p_use > 8
    meta = {"train_problems": a.train, "val_problems": a.val, "samples_per_problem": 4, "steps": a.steps,
            "loss": hist[-5:], "dataset_seconds": round(t_data, 1),
            "tols": "4 per problem, log-uniform in [1e-16, 1e-5]",
            "sizes": "M, N log-uniform in [256, 4096], K log-uniform in [256, 16384]",
            "phi": "U(0,4) for A and for B",
            "labels": "smallest p (s) with E_cw <= tol / 2 on up to 512 x 512 sampled outputs",
            "calibration": "per head, 0.5 logit below the lowest held-out logit whose E_cw at that count > tol",
            "heads": "8 for p > t (t = 1..8), 20 for s > t (t = 1..20)", "margin": 0,
            "val_mean_p_selector": float(p_use.double().mean()), "val_mean_p_bound": float(pb.double().mean()),
            "val_to_scheme2_selector": int(to2.sum()), "val_to_scheme2_bound": int((pb > 8).sum()),
            "val_scheme2_needed": int((pva_d > 8).sum()), "val_mean_p_needed": float(pva_d.double().mean()),
            "val_under_p": int(((p_use < pf) & ~to2).sum()),
            "val_under_p_half_tol": int(((p_use < pva_d) & ~to2).sum()),
            "val_mean_s_selector": float(s_use[to2].double().mean()) if bool(to2.any()) else 0.0,
            "val_mean_s_bound": float(torch.clamp(sb[to2], max=20).double().mean()) if bool(to2.any()) else 0.0,
            "val_mean_s_needed": float(sva_d[to2].double().mean()) if bool(to2.any()) else 0.0,
            "val_under_s": int(((s_use < sf) & to2 & (sf <= 20)).sum()),
            "val_under_s_half_tol": int(((s_use < sva_d) & to2 & (sva_d <= 20)).sum())}
    save(a.out, w, thr, 0, meta)
    print(json.dumps(meta), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
