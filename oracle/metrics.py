"""Error metrics against the double-double reference.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper reports "effective bits", the magnitude of the base-2 exponent of
the relative error, without naming the norm (Sec. V-B).  Reading used here:
* E_cw = max_ij |C - C_ref|_ij / (|A| |B|)_ij  (componentwise, the gate); for
  complex data the real and imaginary parts are scaled separately by the
  magnitude sums of the terms forming them, |Ar||Br| + |Ai||Bi| for the real
  part and |Ar||Bi| + |Ai||Br| for the imaginary part;
* E_nw = ||C - C_ref||_F / ||C_ref||_F          (normwise, reported);
* bits = -log2(E);
* the median over outputs of |C - C_ref| / |C_ref|  (reported).
"""
from __future__ import annotations

import math

import numpy as np


def _abs_product(A, B):
    return np.abs(A) @ np.abs(B)


def e_cw(C, ref_hi, ref_lo, A, B) -> float:
    """Componentwise error scaled by (|A||B|); entries with a zero scale and
    non-finite outputs are left out."""
    C = np.asarray(C)
    if np.iscomplexobj(C) or np.iscomplexobj(A):
        Ar, Ai = np.real(A), np.imag(A)
        Br, Bi = np.real(B), np.imag(B)
        den_re = _abs_product(Ar, Br) + _abs_product(Ai, Bi)
        den_im = _abs_product(Ar, Bi) + _abs_product(Ai, Br)
        err_re = np.abs((C.real - ref_hi.real) - ref_lo.real)
        err_im = np.abs((C.imag - ref_hi.imag) - ref_lo.imag)
        r1 = _ratio(err_re, den_re)
        r2 = _ratio(err_im, den_im)
        return max(r1, r2)
    den = _abs_product(np.asarray(A, np.float64), np.asarray(B, np.float64))
    err = np.abs((C - ref_hi) - ref_lo)
    return _ratio(err, den)


def _ratio(err, den) -> float:
    ok = (den > 0) & np.isfinite(err)
    if not ok.any():
        return 0.0
    return float(np.max(err[ok] / den[ok]))


def e_nw(C, ref_hi, ref_lo) -> float:
    """Frobenius norm of the error over that of the reference (complex
    entries by their modulus)."""
    C = np.asarray(C)
    diff = (C - ref_hi) - ref_lo
    num = np.sqrt(np.sum(np.abs(diff) ** 2))
    den = np.sqrt(np.sum(np.abs(ref_hi + ref_lo) ** 2))
    return float(num / den) if den > 0 else float(num)


def median_rel(C, ref_hi, ref_lo) -> float:
    """Median over the outputs with a nonzero reference of |C - ref| / |ref|."""
    C = np.asarray(C)
    ref = np.asarray(ref_hi) + np.asarray(ref_lo)
    diff = np.abs((C - ref_hi) - ref_lo)
    ok = (np.abs(ref) > 0) & np.isfinite(diff)
    if not ok.any():
        return 0.0
    return float(np.median(diff[ok] / np.abs(ref[ok])))


def bits(err: float) -> float:
    """Effective bits of an error: -log2(err), infinite for an exact result."""
    return math.inf if err <= 0 else -math.log2(err)
