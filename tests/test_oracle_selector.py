"""Pins of the selector reference: analytic gradients against central finite
differences, Adam's first step against its closed form, the histogram
against a brute-force count, and the a-priori bound against the measured
error of the Scheme I oracle."""
import math

import numpy as np

import oracle
import synth
from oracle import selector as sel


def _params(seed):
    r = np.random.default_rng(seed)
    return (r.standard_normal((sel.N_FEAT, sel.HIDDEN)) * 0.3, r.standard_normal(sel.HIDDEN) * 0.1,
            r.standard_normal((sel.HIDDEN, sel.HIDDEN)) * 0.2, r.standard_normal(sel.HIDDEN) * 0.1,
            r.standard_normal((sel.HIDDEN, sel.N_OUT)) * 0.2, r.standard_normal(sel.N_OUT) * 0.1)


def test_backward_matches_finite_differences():
    r = np.random.default_rng(1)
    params = _params(2)
    X = r.random((7, sel.N_FEAT))
    y = sel.ordinal_targets(r.integers(1, 10, 7))
    logits, cache = sel.mlp_forward(params, X)
    grads = sel.mlp_backward(params, cache, logits, y)
    h = 1e-6
    for pi in range(6):
        P = params[pi]
        flat = P.reshape(-1)
        for idx in r.choice(flat.size, min(12, flat.size), replace=False):
            plus = [q.copy() for q in params]
            minus = [q.copy() for q in params]
            plus[pi].reshape(-1)[idx] += h
            minus[pi].reshape(-1)[idx] -= h
            lp = sel.bce_loss(sel.mlp_forward(tuple(plus), X)[0], y)
            lm = sel.bce_loss(sel.mlp_forward(tuple(minus), X)[0], y)
            fd = (lp - lm) / (2 * h)
            an = grads[pi].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 + 1e-5 * abs(fd), (pi, idx, fd, an)


def test_adam_first_step_closed_form():
    """With zero moments, the first bias-corrected step moves every
    parameter by lr * g / (|g| + eps)."""
    params = _params(3)
    r = np.random.default_rng(4)
    grads = tuple(r.standard_normal(p.shape) for p in params)
    zeros = tuple(np.zeros_like(p) for p in params)
    new, m, v = sel.adam_step(params, grads, zeros, zeros, 1, lr=0.01)
    for p0, p1, g in zip(params, new, grads):
        assert np.allclose(p0 - p1, 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)


def test_histogram_brute_force():
    A = synth.phi_matrix(13, 40, 3.0, 5)
    A[2] = 0
    A[4, :7] = 0
    h = sel._hist(A, 1)
    counts = np.zeros(sel.N_BINS)
    for i in range(13):
        nz = [x for x in A[i] if x != 0]
        if not nz:
            continue
        e = max(math.frexp(x)[1] for x in nz)
        for x in nz:
            d = e - math.frexp(x)[1]
            b = max(k for k, edge in enumerate(sel.BIN_EDGES) if d >= edge)
            counts[b] += 1
    assert np.allclose(h, counts / counts.sum(), rtol=0, atol=1e-15)
    c, dmax = sel.deficit_counts(A, 1)
    assert c.tolist() == counts.tolist()
    assert dmax == max(max(math.frexp(x)[1] for x in A[i] if x != 0) - math.frexp(x)[1]
                       for i in range(13) for x in A[i] if x != 0)
    f = sel.features(A, A.T.copy(), 1e-13)
    assert f.shape == (34,) and abs(f[32] - math.log2(40) / 14) < 1e-15 and abs(f[33] - 13 / 16) < 1e-15


def test_deficit_bins_brute_force():
    """Bin of every deficit 0..300 against the edge list read literally."""
    for d in range(301):
        b = max(k for k, edge in enumerate(sel.BIN_EDGES) if d >= edge)
        assert sel.deficit_bin(d) == b
        A = np.array([[1.0, math.ldexp(1.0, -d)]])
        assert sel.deficit_counts(A, 1)[0].tolist() == [2 if (k == 0 and b == 0) else int(k == 0) + int(k == b)
                                                        for k in range(sel.N_BINS)]


def test_nonfinite_lines_and_columns_are_skipped():
    A = synth.phi_matrix(6, 9, 2.0, 3)
    A[1, 4] = np.inf
    A[3, 0] = np.nan
    c_rows, _ = sel.deficit_counts(A, 1)
    keep = np.delete(A, [1, 3], axis=0)
    assert c_rows.tolist() == sel.deficit_counts(keep, 1)[0].tolist() and c_rows.sum() == 4 * 9
    c_cols, _ = sel.deficit_counts(A, 0)
    keepc = np.delete(A, [0, 4], axis=1)
    assert c_cols.tolist() == sel.deficit_counts(keepc, 0)[0].tolist() and c_cols.sum() == 6 * 7


def test_bound_holds_on_oracle_errors():
    """The a-priori bound is never below the measured error."""
    for phi, seed in ((0.5, 1), (1.0, 2), (2.0, 3)):
        A = synth.phi_matrix(20, 64, phi, 10 + seed)
        B = synth.phi_matrix(64, 18, phi, 20 + seed)
        hi, lo = oracle.gemm_dd(A, B)
        ra, rb = sel.max_deficit(A, 1), sel.max_deficit(B, 0)
        for p in range(1, 9):
            err = oracle.metrics.e_cw(oracle.s1_dgemm(A, B, p), hi, lo, A, B)
            assert err <= sel.bound(p, ra, rb), (phi, p, err, sel.bound(p, ra, rb))


def test_scheme2_bound_holds_on_oracle_errors():
    """The Scheme II bound is never below the measured error; with a narrow
    exponent range (phi = 0.5) it is also within 2^20 of it above the
    rounding floor, so a dropped or misplaced term shows up either way."""
    from oracle import scheme2 as s2
    for phi, seed, K in ((0.5, 1, 64), (1.0, 2, 100), (2.0, 3, 37), (3.0, 4, 200)):
        A = synth.phi_matrix(12, K, phi, 30 + seed)
        B = synth.phi_matrix(K, 9, phi, 40 + seed)
        hi, lo = oracle.gemm_dd(A, B)
        ra, rb = sel.max_deficit(A, 1), sel.max_deficit(B, 0)
        for s in (4, 6, 8, 10, 12, 14, 16):
            err = oracle.metrics.e_cw(s2.s2_dgemm(A, B, s), hi, lo, A, B)
            bnd = sel.bound_s2(s, ra, rb, K)
            assert err <= bnd, (phi, s, err, bnd)
            if phi == 0.5 and err > 1e-14:
                assert bnd < err * 2.0 ** 20, (phi, s, err, bnd)


def test_complex_scheme2_bound_holds_on_oracle_3m_errors():
    """The 3M bound (part deficits plus one) is never below the complex E_cw
    of the oracle's 3M product, including parts of very different size
    within an entry and the re ~ im cancellation case, and with a narrow
    exponent range it stays within 2^21 of the error above the rounding
    floor; the part deficits on a hand-evaluated case."""
    from oracle import scheme2 as s2
    rng = np.random.default_rng(7)
    cases = []
    for phi, seed, K in ((0.5, 1, 40), (1.0, 2, 64), (2.5, 3, 23)):
        cases.append((synth.complex_phi_matrix(10, K, phi, 50 + seed, 60 + seed),
                      synth.complex_phi_matrix(K, 7, phi, 70 + seed, 80 + seed)))
    X = rng.standard_normal((8, 30))
    cases.append((X + 1j * X * (1 + 2.0 ** -30), synth.complex_phi_matrix(30, 6, 1.0, 90, 91)))
    A = synth.complex_phi_matrix(9, 33, 0.5, 92, 93)
    A.imag *= 2.0 ** -20  # imaginary parts far below the real parts of the same entries
    cases.append((A, synth.complex_phi_matrix(33, 5, 0.5, 94, 95)))
    for A, B in cases:
        K = A.shape[1]
        hi, lo = oracle.zgemm_dd(A, B)
        ra, rb = sel.complex_max_deficits(A, B)
        for s in (6, 8, 10, 12, 14, 16):
            err = oracle.metrics.e_cw(s2.z3m_gemm(A, B, s), hi, lo, A, B)
            bnd = sel.bound_s2(s, ra + 1, rb + 1, K)
            assert err <= bnd, (s, err, bnd)
            if A is cases[0][0] and err > 1e-14:
                assert bnd < err * 2.0 ** 21, (s, err, bnd)
    # parts 1, 0.25, 2^-10 in a row: deficits 0, 2, 10; a column of 1j and 0.5: 0, 1
    Ah = np.array([[1 + 0.25j, 2.0 ** -10 * 1j], [0.0, 3.0]])
    Bh = np.array([[1j, 0.0], [0.5, 0.0]])
    assert sel.complex_max_deficits(Ah, Bh) == (10, 1)
    A, B = cases[0]
    prev = 0
    for tol in (1e-4, 1e-8, 1e-12, 1e-15, 1e-17):
        s = sel.s_bound_complex(A, B, tol)
        assert s >= prev
        prev = s
    assert sel.s_bound_complex(A, B, 1e-17) == 21


def test_s_bound_monotone_and_consistent():
    A = synth.phi_matrix(10, 50, 1.0, 1)
    B = synth.phi_matrix(50, 8, 1.0, 2)
    prev = 0
    for tol in (1e-3, 1e-6, 1e-9, 1e-12, 1e-15, 1e-17):
        s = sel.s_bound(A, B, tol)
        assert s >= prev
        prev = s
        if s <= 20:
            ra, rb = sel.max_deficit(A, 1), sel.max_deficit(B, 0)
            assert sel.bound_s2(s, ra, rb, 50) <= tol
            if s > 1:
                assert sel.bound_s2(s - 1, ra, rb, 50) > tol
    assert sel.s_bound(A, B, 1e-17) == 21  # below the rounding floor


def test_predict_and_targets():
    y = sel.ordinal_targets(np.array([1, 3, 9]), np.array([21, 1, 5]))
    assert y.shape == (3, sel.N_OUT)
    assert y[0, :8].tolist() == [0] * 8 and y[1, :8].tolist() == [1, 1, 0, 0, 0, 0, 0, 0] and y[2, :8].tolist() == [1] * 8
    assert y[0, 8:].tolist() == [1] * 20 and y[1, 8:].tolist() == [0] * 20
    assert y[2, 8:].tolist() == [1, 1, 1, 1] + [0] * 16  # s = 5: heads s > 1 .. s > 4
    logits = np.where(y > 0, 5.0, -5.0)
    p, s = sel.predict(logits)
    assert p.tolist() == [1, 3, 9] and s.tolist() == [21, 1, 5]
    p, s = sel.predict(logits, margin=1)
    assert p.tolist() == [2, 4, 9] and s.tolist() == [21, 2, 6]
    # per-head thresholds: raising one head's threshold above its sigmoid drops exactly that head
    thr = np.full(sel.N_OUT, 0.5)
    thr[1] = 0.9999  # head "p > 2" of the second sample (sigmoid(5) = 0.9933) no longer counts
    p, s = sel.predict(logits, thr)
    assert p.tolist() == [1, 2, 8] and s.tolist() == [21, 1, 5]
    assert sel.predict_p(logits).tolist() == [1, 3, 9]


def test_decision_rule():
    # in range with a network: the smaller of the network and the bound
    assert sel.decide(5, 12, 7, 16, True) == (1, 5)
    assert sel.decide(8, 12, 6, 16, True) == (1, 6)
    # Scheme I infeasible: Scheme II at the smaller count
    assert sel.decide(9, 12, 9, 16, True) == (2, 12)
    assert sel.decide(9, 18, 9, 16, True) == (2, 16)
    # out of range or no network: the bounds alone
    assert sel.decide(3, 4, 7, 16, False) == (1, 7)
    assert sel.decide(9, 4, 9, 16, True, have_net=False) == (2, 16)
    # nothing proven: the most accurate Scheme II
    assert sel.decide(9, 21, 9, 21, False) == (2, 20)


def test_forward_on_a_hand_evaluated_network():
    """x = (3, 1, 2, 0, ...): layer 1 gives z = (2*3 - 1, 2 - 5) = (5, -3) ->
    ReLU (5, 0); layer 2 gives (0.5*5 + 1, 7*0 - 1) = (3.5, -1) -> (3.5, 0);
    head t (t = 0..7) is 3.5 t + 0.25.  A missing bias, a missing ReLU or a
    transposed weight changes some head."""
    W1 = np.zeros((sel.N_FEAT, sel.HIDDEN))
    b1 = np.zeros(sel.HIDDEN)
    W2 = np.zeros((sel.HIDDEN, sel.HIDDEN))
    b2 = np.zeros(sel.HIDDEN)
    W3 = np.zeros((sel.HIDDEN, sel.N_OUT))
    b3 = np.full(sel.N_OUT, 0.25)
    W1[0, 0], W1[1, 0], W1[2, 1], b1[1] = 2.0, -1.0, 1.0, -5.0
    W2[0, 0], b2[0], W2[1, 1], b2[1] = 0.5, 1.0, 7.0, -1.0
    W3[0, :] = np.arange(sel.N_OUT)
    X = np.zeros((1, sel.N_FEAT))
    X[0, :3] = (3.0, 1.0, 2.0)
    out, _ = sel.mlp_forward((W1, b1, W2, b2, W3, b3), X)
    assert np.array_equal(out[0], 3.5 * np.arange(sel.N_OUT) + 0.25)
