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
* a plain fp64 MLP 34 -> 64 -> 64 -> 8 (ReLU), ordinal heads z_t ~ P(p > t),
  its binary cross-entropy loss, analytic backward pass and one Adam step.
"""
from __future__ import annotations

import math

import numpy as np

# lower edges of the 16 deficit bins
BIN_EDGES = (0, 1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 256)
N_BINS = len(BIN_EDGES)
N_FEAT = 2 * N_BINS + 2
HIDDEN = 64
N_OUT = 8


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


# -------------------------------------------------------------------- MLP

def mlp_forward(params, X):
    """params = (W1, b1, W2, b2, W3, b3) with W as [in][out]; X [n][34].
    Returns logits [n][8] and the cache for backward."""
    W1, b1, W2, b2, W3, b3 = params
    z1 = X @ W1 + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2 + b2
    h2 = np.maximum(z2, 0.0)
    out = h2 @ W3 + b3
    return out, (X, z1, h1, z2, h2)


def ordinal_targets(p: np.ndarray) -> np.ndarray:
    """y[n][t-1] = 1 if p > t (t = 1..8)."""
    p = np.asarray(p).reshape(-1, 1)
    t = np.arange(1, N_OUT + 1).reshape(1, -1)
    return (p > t).astype(np.float64)


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


def predict_p(logits, threshold: float = 0.5, margin: int = 0) -> np.ndarray:
    """p = 1 + #{t : sigmoid(z_t) > threshold} + margin, capped at 9."""
    sig = 1.0 / (1.0 + np.exp(-np.asarray(logits)))
    return np.minimum(1 + (sig > threshold).sum(axis=1) + margin, 9)
