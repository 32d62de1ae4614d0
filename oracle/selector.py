"""Reference computations for the learned slice-count selector.

TEST INFRASTRUCTURE ONLY (see the package docstring).  The paper has no
selector: it names automatic dynamic precision (a runtime estimate of the
slice count) as missing from its implementation (Sec. VI).  These functions
define what the library's GPU kernels must compute, so that the kernels can
be checked:

* features(A, B, tol): 34 numbers -- the fraction of nonzero entries of A
  (resp. B) in each of 16 bins of the exponent deficit e_i - expo(a_ik)
  relative to the row (column) exponent, log2(K) / 14 and -log10(tol) / 16;
* p_bound(A, B, tol): the smallest p whose a-priori componentwise error
  bound for the balanced 8-bit slices is below tol (9 = none up to 8);
* a plain fp64 MLP 34 -> 64 -> 64 -> 28 (ReLU) with ordinal heads: z_t ~
  P(p > t) for the Scheme I slice count (t = 1..8, heads 0..7) and z_t ~
  P(s > t) for the Scheme II modulus count (t = 1..20, heads 8..27), its
  binary cross-entropy loss, analytic backward pass and one Adam step, and
  the decision rule (per-head thresholds plus a margin).
"""
from __future__ import annotations

import math

import numpy as np

# lower edges of the 16 deficit bins
BIN_EDGES = (0, 1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 256)
N_BINS = len(BIN_EDGES)
N_FEAT = 2 * N_BINS + 2
HIDDEN = 64
P_HEADS = 8    # Scheme I: p > t, t = 1..8
S_HEADS = 20   # Scheme II: s > t, t = 1..20
N_OUT = P_HEADS + S_HEADS


def deficit_bin(d: int) -> int:
    b = 0
    for i, edge in enumerate(BIN_EDGES):
        if d >= edge:
            b = i
    return b


def deficit_counts(X, axis: int):
    """Integer counts of the exponent deficits per bin and the largest
    deficit.  Deficits are taken against the largest exponent of each row
    (axis=1) or column (axis=0) over its nonzero entries; zero entries are
    not counted, and a row (column) holding a non-finite entry contributes
    nothing (its outputs are not finite whatever p is)."""
    X = np.asarray(X, np.float64)
    if X.size == 0:
        return np.zeros(N_BINS, np.int64), 0
    fin = np.isfinite(X)
    ok_line = fin.all(axis=axis, keepdims=True)
    nz = fin & (X != 0) & ok_line
    _, ex = np.frexp(np.where(nz, X, 1.0))
    ex = np.where(nz, ex, np.iinfo(np.int32).min).astype(np.int64)
    emax = ex.max(axis=axis, keepdims=True)
    d = (emax - ex)[nz]
    bins = np.searchsorted(np.asarray(BIN_EDGES), d, side="right") - 1
    counts = np.bincount(bins, minlength=N_BINS).astype(np.int64)
    return counts, int(d.max()) if d.size else 0


def _hist(X, axis: int) -> np.ndarray:
    """Fractions of the counted entries per deficit bin."""
    counts, _ = deficit_counts(X, axis)
    n = counts.sum()
    return counts / n if n else counts.astype(np.float64)


def max_deficit(X, axis: int) -> int:
    return deficit_counts(X, axis)[1]


def features(A, B, tol: float) -> np.ndarray:
    K = np.asarray(A).shape[1]
    f = np.concatenate([_hist(A, 1), _hist(B, 0),
                        [math.log2(max(K, 1)) / 14.0, -math.log10(tol) / 16.0]])
    return f.astype(np.float64)


def bound(p: int, ra: int, rb: int) -> float:
    """A-priori componentwise error bound for p balanced slices (8p-2 bits,
    rounding error <= 2^-(8p-1) of the row/column scale), for entries at most
    ra (rb) exponent steps below their row (column) maximum:
      each term: 2^-(8p-1) (2^(ra+1) + 2^(rb+1)) + 2^-2(8p-1) 2^(ra+rb+2)
      + dropped slice pairs (at most p-1 pairs per diagonal d >= p, each
        below 128^2 2^(-12-8d)): (p-1) 1.01 2^(2-8p) 2^(ra+rb+2),
    plus the final rounding 2^-53."""
    if ra + rb + 2 > 1000:  # beyond any tolerance <= 1
        return math.inf
    a = 2.0 ** (-(8 * p - 1)) * (2.0 ** (ra + 1) + 2.0 ** (rb + 1))
    a += 2.0 ** (-2 * (8 * p - 1)) * 2.0 ** (ra + rb + 2)
    a += (p - 1) * 1.01 * 2.0 ** (2 - 8 * p) * 2.0 ** (ra + rb + 2)
    return a + 2.0 ** -53


def p_bound(A, B, tol: float) -> int:
    ra, rb = max_deficit(A, 1), max_deficit(B, 0)
    for p in range(1, 9):
        if bound(p, ra, rb) <= tol:
            return p
    return 9


def bound_s2(s: int, ra: int, rb: int, K: int) -> float:
    """A-priori componentwise error bound of Scheme II with s moduli for
    entries at most ra (rb) exponent steps below their row (column) maximum
    (Sec. II-C.2 with the norm-bound scales): the scale exponent nb exceeds
    the row maximum by at most d = ceil(ceil(log2 K) / 2), an entry r steps
    below the maximum is at least 2^(e-r-1), so truncating it at 2^(nb-T)
    costs at most 2^(r+d+1-T) relative; per product term the two relative
    errors and their product, then the final rounding (the CRT is exact)."""
    from .scheme2 import targets
    ta, tb = targets(s)
    d = (max(int(K), 1) - 1).bit_length()  # ceil(log2 K)
    d = (d + 1) // 2
    ea, eb = ra + d + 1 - ta, rb + d + 1 - tb
    if max(ea, eb, ea + eb) > 1000:
        return math.inf
    return 2.0 ** ea + 2.0 ** eb + 2.0 ** (ea + eb) + 2.0 ** -53


def s_bound(A, B, tol: float) -> int:
    """Smallest s in [1, 20] whose bound is <= tol (21 = none)."""
    ra, rb = max_deficit(A, 1), max_deficit(B, 0)
    K = np.asarray(A).shape[1]
    for s in range(1, 21):
        if bound_s2(s, ra, rb, K) <= tol:
            return s
    return 21


def complex_max_deficits(A, B):
    """The largest exponent deficit of a nonzero real or imaginary part below
    the largest part exponent of its row of A (column of B): the real
    deficits of [Re A, Im A] by rows and of [Re B; Im B] by columns."""
    A = np.asarray(A, np.complex128)
    B = np.asarray(B, np.complex128)
    ra = max_deficit(np.concatenate([A.real, A.imag], axis=1), 1)
    rb = max_deficit(np.concatenate([B.real, B.imag], axis=0), 0)
    return ra, rb


def s_bound_complex(A, B, tol: float) -> int:
    """Smallest s in [1, 20] whose Scheme II bound for the 3M product is <=
    tol (21 = none): the real bound with each part deficit one more, since the
    shared per-row (per-column) scale is taken from |re| + |im| < 2^(max(expo
    re, expo im) + 1) -- an entry part r steps below the row's largest part
    exponent lies r + 1 steps below the complex entry exponent the scale
    uses.  Each part of the result is a sum of real products whose
    magnitudes are the scale of that part in the complex E_cw, so the
    per-term relative errors carry over."""
    ra, rb = complex_max_deficits(A, B)
    K = np.asarray(A).shape[1]
    for s in range(1, 21):
        if bound_s2(s, ra + 1, rb + 1, K) <= tol:
            return s
    return 21


# -------------------------------------------------------------------- MLP

def mlp_forward(params, X):
    """params = (W1, b1, W2, b2, W3, b3) with W as [in][out]; X [n][34].
    Returns logits [n][28] and the cache for backward."""
    W1, b1, W2, b2, W3, b3 = params
    z1 = X @ W1 + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2 + b2
    h2 = np.maximum(z2, 0.0)
    out = h2 @ W3 + b3
    return out, (X, z1, h1, z2, h2)


def ordinal_targets(p: np.ndarray, s: np.ndarray = None) -> np.ndarray:
    """y[n][t-1] = 1 if p > t (t = 1..8) and y[n][7+t] = 1 if s > t
    (t = 1..20); p = 9 means no slice count up to 8 meets the tolerance, s =
    21 no modulus count up to 20 (s defaults to 21)."""
    p = np.asarray(p).reshape(-1, 1)
    s = np.full(p.shape, 21) if s is None else np.asarray(s).reshape(-1, 1)
    tp = np.arange(1, P_HEADS + 1).reshape(1, -1)
    ts = np.arange(1, S_HEADS + 1).reshape(1, -1)
    return np.concatenate([(p > tp), (s > ts)], axis=1).astype(np.float64)


def bce_loss(logits, y) -> float:
    """Mean binary cross-entropy over samples and heads (stable form)."""
    l = np.maximum(logits, 0) - logits * y + np.log1p(np.exp(-np.abs(logits)))
    return float(l.mean())


def mlp_backward(params, cache, logits, y):
    """Gradients of bce_loss with respect to every parameter."""
    W1, b1, W2, b2, W3, b3 = params
    X, z1, h1, z2, h2 = cache
    n = X.shape[0]
    sig = 1.0 / (1.0 + np.exp(-logits))
    g_out = (sig - y) / (n * N_OUT)
    gW3 = h2.T @ g_out
    gb3 = g_out.sum(axis=0)
    g_h2 = g_out @ W3.T
    g_z2 = g_h2 * (z2 > 0)
    gW2 = h1.T @ g_z2
    gb2 = g_z2.sum(axis=0)
    g_h1 = g_z2 @ W2.T
    g_z1 = g_h1 * (z1 > 0)
    gW1 = X.T @ g_z1
    gb1 = g_z1.sum(axis=0)
    return (gW1, gb1, gW2, gb2, gW3, gb3)


def adam_step(params, grads, m, v, t: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (bias-corrected), returning (params, m, v)."""
    out_p, out_m, out_v = [], [], []
    for p, g, mm, vv in zip(params, grads, m, v):
        mm = beta1 * mm + (1 - beta1) * g
        vv = beta2 * vv + (1 - beta2) * g * g
        mh = mm / (1 - beta1 ** t)
        vh = vv / (1 - beta2 ** t)
        out_p.append(p - lr * mh / (np.sqrt(vh) + eps))
        out_m.append(mm)
        out_v.append(vv)
    return tuple(out_p), tuple(out_m), tuple(out_v)


def predict(logits, thresholds=0.5, margin: int = 0):
    """The network's counts: p_net = 1 + #{t : sigmoid(z_t) > thr_t over the
    Scheme I heads} + margin, capped at 9, and s_net the same over the
    Scheme II heads, capped at 21.  thresholds: one value or one per head."""
    sig = 1.0 / (1.0 + np.exp(-np.asarray(logits, np.float64)))
    thr = np.broadcast_to(np.asarray(thresholds, np.float64), (N_OUT,))
    up = sig > thr.reshape(1, -1)
    p = np.minimum(1 + up[:, :P_HEADS].sum(axis=1) + margin, 9)
    s = np.minimum(1 + up[:, P_HEADS:].sum(axis=1) + margin, 21)
    return p, s


def predict_p(logits, threshold: float = 0.5, margin: int = 0) -> np.ndarray:
    """The Scheme I count alone (see predict)."""
    return predict(logits, threshold, margin)[0]


def decide(p_net: int, s_net: int, p_b: int, s_b: int, in_range: bool, have_net: bool = True):
    """The library's decision from the network counts and the a-priori
    bounds: p = min(p_net, p_bound) (the bound alone without a network or
    outside the training range); Scheme I with p while p <= 8, else Scheme II
    with s = min(s_net, s_bound) (the bound alone likewise), s = 20 when no
    count up to 20 is proven.  Returns (scheme, count)."""
    use_net = have_net and in_range
    p = min(p_net, p_b) if use_net else p_b
    if p <= 8:
        return 1, p
    s = min(s_net, s_b) if use_net else s_b
    return 2, min(s, 20)
